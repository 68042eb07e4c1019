#!/usr/bin/env python3
"""Benchmark of the NPF hot path on one MI355X.

One step = one pass of the whole hot path over the workload: plan (Alg. 1 block sizing),
upper-index contraction, the lower-index chain, divisor / division, reduction to P_M
for every order, and the NPF assembly (Alg. 2), with inputs already resident in HBM.

Default workload: n = 200 states, orders 2-4, dense derivative tensors generated on the
device (never stored).  Prints ONE JSON line: modal tensor entries per second (sum over
orders of n * U_M symmetric-unique entries of the full NPF per step / step time) for the
selected precision (split-BF16), the same for the FP32 and plain FP64 GPU paths, the error
of each against the CPU FP64 oracle (pooled, per output mode and max-entry), the roofline of
the dominant kernel (timed live with HIP events on its launch stream) and the oracle's own
rate on the host cores.  A real system's modes come in conjugate pairs: by default one
mode of each pair is computed and the other filled by conjugation (--no-conj computes all).
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
# Dense matrix-core peaks of MI355X for the engine each path runs on: FP64, FP64 (the FP32
# path forms exact FP32 products and accumulates in FP64 on the FP64 matrix cores), BF16.
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 78.6, "bf16x3": 2500.0}
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


# Budget of the generated-versus-stored pair: the stored order-4 tensor of 200 states takes
# 110 GB beside the workspace, so both legs run under 140 GB (blocks of 16 modes).
SOURCE_PAIR_BUDGET = 140 << 30


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
    """(algorithmic flops, algorithmic HBM bytes, bound, uses MFMA) of one launch of a
    kernel, averaged over the plan's blocks, from the shapes (a complex multiply-add counts
    8 flops, real x complex 4).  J is the mean number of computed modes per block: a narrow
    last block (or padding to 16 modes) is not algorithmic work."""
    n, U = sysm.n, plan.unique_tuples
    J = plan.computed_modes / max(1, plan.n_blocks)
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


def time_path(sysm, s, precision, steps, warmup, device, profile, budget=0, progress=False,
              conj=True):
    """Time `steps` steps on a dedicated stream (graph replay after the first call), then
    run `profile` more steps eagerly with HIP events around every kernel launch.  With
    `progress` (multi-second steps) every step is synchronised and logged.  With `conj` the
    plan computes one mode of each conjugate pair and fills the other (a real system)."""
    import torch
    from paper_2509_08968_amd import binding as B

    n, N = s.n, s.order_max
    P = torch.empty((N - 1, n, n), dtype=torch.complex128, device=device)
    npf = torch.empty((n, n), dtype=torch.complex128, device=device)
    conj_of = B.conj_pairs(s.lam) if conj else None
    mk = lambda: B.Plan(n, N, precision, s.eps, s.tau, s.delta, budget_bytes=budget,
                        support_max=s.support_max, conj_of=conj_of)
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
        for i in range(profile):
            p = mk()
            p.profile(True)            # eager launches, an event pair around each kernel
            step(p)
            plans.append(p)
            if progress:
                torch.cuda.synchronize()
                log(f"[bench] {precision} profiled step {i + 1}/{steps} done")
        e3.record(stream)
        torch.cuda.synchronize()
        out["eager_ms_per_step"] = e2.elapsed_time(e3) / profile
        out["profile_steps"] = profile
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


def err_summary(got, ref):
    """Errors of a result whose rows are output modes: pooled relative Frobenius error,
    the largest per-mode relative error (each row against its own norm) and the max-entry
    error max|got - ref| / max|ref|."""
    import numpy as np
    got, ref = np.atleast_2d(got), np.atleast_2d(ref)
    d = np.linalg.norm(got - ref, axis=1)
    nb = np.linalg.norm(ref, axis=1)
    per = d / np.where(nb > 0, nb, 1.0)
    return {"pooled": rel(got, ref), "per_mode_max": float(per.max()),
            "max_entry": float(np.abs(got - ref).max() / np.abs(ref).max())}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Threads the oracle may use on this host: the CPUs this process may run on, capped by
    OMP_NUM_THREADS when it is set (the machine's CPU share)."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        cores = min(cores, int(env))
    return max(1, cores)


def cpu_baseline(s, entries, target_s=10.0):
    """The oracle as it stands, timed on this host's cores over a bounded sample, scaled to
    modal entries per second: all the threads this host gives the process, and one thread.
    Small systems: the full workload repeated until about target_s seconds have passed.
    Large systems (the oracle takes minutes per mode at order 4): output mode 0 of every
    order with all threads, mode 0 of the orders below 4 with one thread."""
    import oracle
    cores = host_threads()

    def run(threads, orders, modes):
        t0, reps, done = time.perf_counter(), 0, 0
        while True:
            for M in orders:
                oracle.sym(s, M, modes=modes, nthreads=threads)
                done += (s.n if modes is None else len(modes)) * math.comb(s.n + M - 1, M)
            reps += 1
            el = time.perf_counter() - t0
            if modes is not None or el >= target_s or reps >= 1000:
                return done, el, reps

    if s.n > 64:
        done, el, _ = run(cores, s.orders, [0])
        low = [M for M in s.orders if M < 4]
        d1, e1, _ = run(1, low, [0])
        return {"value": done / el, "unit": "modal entries/s", "cores": cores, "kind": "oracle",
                "cpu_model": cpu_model(),
                "sample": f"output mode 0 of orders {s.orders}: {done} entries in {el:.1f} s, "
                          f"packed-symmetric FP64 oracle with {cores} OpenMP threads",
                "one_thread": {"value": d1 / e1, "cores": 1,
                               "sample": f"output mode 0 of orders {low}: {d1} entries in "
                                         f"{e1:.1f} s, one thread"}}
    done, el, reps = run(cores, s.orders, None)
    d1, e1, r1 = run(1, s.orders, None)
    return {"value": done / el, "unit": "modal entries/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"full workload (all output modes, orders {s.orders}) x {reps} repeats, "
                      f"{el:.1f} s, packed-symmetric FP64 oracle with {cores} OpenMP threads",
            "one_thread": {"value": d1 / e1, "cores": 1,
                           "sample": f"the same x {r1} repeats, {e1:.1f} s, one thread"}}


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
            e = err_summary(got, ref)
            cur = errs.setdefault(f"P{M}", {k: 0.0 for k in e})
            for k, v in e.items():
                cur[k] = max(cur[k], v)

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

    # Per-system runs: each system alone through npf_run -- split-BF16 with eager launches
    # and replayed graphs, and plain FP64 (replayed graphs) as the batched path's baseline.
    solo = None
    if not args.no_solo:
        del ws
        torch.cuda.empty_cache()

        def solo_leg(prec, graph):
            big = max(B.Plan(s.n, s.order_max, prec, support_max=s.support_max).workspace_bytes
                      for s in ss)
            wsolo = torch.empty(big, dtype=torch.uint8, device=device)
            rates, total = [], 0.0
            for q, s in enumerate(ss):
                plan = B.Plan(s.n, s.order_max, prec, s.eps, s.tau, s.delta,
                              support_max=s.support_max, graph=graph)
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
            del wsolo
            torch.cuda.empty_cache()
            rates = np.asarray(rates)
            return {"sum_ms": total, "batch_speedup": total / ms,
                    "entries_per_s_min": float(rates.min()),
                    "entries_per_s_median": float(np.median(rates)),
                    "entries_per_s_max": float(rates.max())}

        solo = {"bf16x3_eager": solo_leg("bf16x3", False), "bf16x3_graph": solo_leg("bf16x3", True)}
        solo["batching_speedup"] = solo["bf16x3_eager"]["batch_speedup"]
        fp64 = solo_leg("fp64", True)
        e64 = {}
        for q in picks:                     # the FP64 results of the sampled systems
            s = ss[q]
            modes = sorted({0, s.n // 2 + 1, s.n - 1})
            for M in s.orders:
                e = err_summary(P[q][M - 2].cpu().numpy()[modes],
                                oracle.sym(s, M, modes=modes)["P"])
                cur = e64.setdefault(f"P{M}", {k: 0.0 for k in e})
                for k, v in e.items():
                    cur[k] = max(cur[k], v)
        fp64["rel_err"] = e64
        solo["fp64_graph"] = fp64
        log(f"[bench] solo: bf16x3 eager {solo['bf16x3_eager']['sum_ms']:.3f} ms, graph "
            f"{solo['bf16x3_graph']['sum_ms']:.3f} ms, fp64 graph {fp64['sum_ms']:.3f} ms; "
            f"batch {ms:.3f} ms")

    cpu = None
    if not args.no_cpu_baseline:
        cores = host_threads()
        small = [ss[int(i)] for i in order[:24]]
        t0 = time.perf_counter()
        done = 0
        for s in small:
            for M in s.orders:
                oracle.sym(s, M, nthreads=cores)
                done += s.n * math.comb(s.n + M - 1, M)
        el = time.perf_counter() - t0
        cpu = {"value": done / el, "unit": "modal entries/s", "cores": cores, "kind": "oracle",
               "cpu_model": cpu_model(),
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


def interaction_leg(s, sysm, precision, budget, conj, device, refP, modes):
    """npf_run_interaction on the workload (the NPFs and the interaction factors of
    eqs. (8)-(9), two passes of the chain): one warm call, one timed call; errors against the
    oracle when the reference holds every mode's P (n <= 64)."""
    import numpy as np
    import torch

    import oracle
    from paper_2509_08968_amd import binding as B
    n, N = s.n, s.order_max
    plan = B.Plan(n, N, precision, s.eps, s.tau, s.delta, budget_bytes=budget,
                  support_max=s.support_max, conj_of=B.conj_pairs(s.lam) if conj else None)
    ws = plan.workspace(device)
    Q = torch.empty((N - 1, n, n), dtype=torch.complex128, device=device)
    P = torch.empty((N - 1, n, n), dtype=torch.complex128, device=device)
    npf = torch.empty((n, n), dtype=torch.complex128, device=device)
    st = torch.cuda.Stream(device=device)
    plan.run_interaction(sysm.tensors, sysm.U, sysm.V, sysm.lam, ws, Q, P, npf, st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    plan.run_interaction(sysm.tensors, sysm.U, sysm.V, sysm.lam, ws, Q, P, npf, st)
    e1.record(st)
    torch.cuda.synchronize()
    out = {"ms_per_step": e0.elapsed_time(e1), "passes": 2,
           "modal_entries_per_pass": plan.modal_entries, "timing": "one eager call after a warm one"}
    if len(modes) == n:
        ref = oracle.interaction(s, Ps={M: np.asarray(refP[M]) for M in s.orders})
        out["rel_err"] = {f"p{M}": err_summary(Q[M - 2].cpu().numpy().T, ref[M].T)
                          for M in s.orders}
    else:
        out["rel_err"] = None
        out["parity"] = "tests/test_gpu_interaction.py (the oracle needs every mode's P)"
    plan.close()
    del ws
    torch.cuda.empty_cache()
    return out


def source_pair(s, sysm, precision, conj, device, budget, errors):
    """The workload with its hash-generated tensors generated inside the upper-index
    contraction (as benchmarked) and stored in HBM (materialised once with npf_hash_fill,
    outside the timed region, and read as dense tensors), both under the same budget so
    that the stored tensors fit beside the workspace: one warm step and one timed step each."""
    import torch
    from paper_2509_08968_amd import binding as B
    if not s.hashed:
        return None
    stored, bufs = [], []
    for t in sysm.tensors:
        if t.kind != B.SRC_HASH:
            stored.append(t)
            continue
        M = t.order
        UM = math.comb(s.n + M - 1, M)
        buf = torch.empty(s.n * UM, dtype=torch.float64, device=device)
        B.hash_fill(s.n, M, t.desc.seed, t.desc.scale, 0, s.n, buf)
        bufs.append(buf)
        stored.append(B.DeviceTensor(M, B.SRC_DENSE, {"values": buf},
                                     B.NpfTensor(B.SRC_DENSE, M, buf.data_ptr(), None, None, None,
                                                 0, 0)))
    torch.cuda.synchronize()
    out = {"budget_bytes": budget, "stored_tensor_bytes": sum(8 * b.numel() for b in bufs)}
    for name, tens in (("generated", sysm.tensors), ("stored", stored)):
        dev = B.DeviceSystem(sysm.n, sysm.lam, sysm.U, sysm.V, tens, sysm.orders, sysm.support_max)
        r = time_path(dev, s, precision, 1, 1, device, 0, budget, s.n > 128, conj)
        out[name] = {"ms_per_step": r["ms_per_step"], "value": r["plan"].modal_entries / (r["ms_per_step"] * 1e-3),
                     "rel_err": errors(r), "block_modes": r["plan"].block_modes,
                     "blocks": r["plan"].n_blocks}
        r["plan"].close()
        del r
        torch.cuda.empty_cache()
    del bufs, stored
    torch.cuda.empty_cache()
    return out


def taylor_leg(device, n=200):
    """npf_taylor_fill (the numerical Taylor expansion of Alg. 1 on the device) for a seeded
    polynomial field of n states with terms of degrees 1-4 about a nonzero x*: all rows of
    A_3 (checked element by element against the oracle's binomial expansion) and a 16-row
    batch of A_4, each timed over three calls after a warm one."""
    import numpy as np
    import torch

    import oracle
    from paper_2509_08968_amd import binding as B
    from paper_2509_08968_amd import inputs as I
    rng = np.random.default_rng(I.BASE_SEED + 77)
    field = I.poly_field(n, [2, 3, 4], I.BASE_SEED + 78, terms_per_eq=6,
                         x_eq=rng.standard_normal(n) * 0.3)
    poly = B.DevicePoly(field, device)
    st = torch.cuda.Stream(device=device)
    res = {"n": n, "terms": int(len(field["coef"])), "max_degree": 4}
    for M, rows in ((3, n), (4, 16)):
        UM = math.comb(n + M - 1, M)
        buf = torch.empty(rows * UM, dtype=torch.float64, device=device)
        B.taylor_fill(poly, M, 0, rows, buf, st)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(3):
            B.taylor_fill(poly, M, 0, rows, buf, st)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        r = {"rows": rows, "entries": rows * UM, "ms_per_call": ms,
             "entries_per_s": rows * UM / (ms * 1e-3),
             "write_GBps": 8 * rows * UM / (ms * 1e-3) / 1e9}
        r["write_frac_of_hbm_peak"] = r["write_GBps"] / HBM_GBPS
        if M == 3:
            ref = oracle.poly_tensor(field, n, M)
            got = buf.cpu().numpy().reshape(rows, UM)
            r["max_abs_err_over_max"] = float(np.abs(got - ref).max() / max(1.0, np.abs(ref).max()))
            del ref, got
        res[f"A{M}"] = r
        del buf
        torch.cuda.empty_cache()
    return res


DEFAULT_WORKLOAD = "n200-o4-dense-hash"


def leg_counts(args, s, which):
    """Timed and warmup steps of a comparison leg: as given, else the main leg's for steps
    of milliseconds and one timed step without warmup for the multi-second n > 128 steps."""
    st = getattr(args, f"{which}_steps")
    wu = getattr(args, f"{which}_warmup")
    big = s.n > 128
    return (st if st is not None else (1 if big else args.steps),
            wu if wu is not None else (0 if big else args.warmup))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-conj", action="store_true",
                    help="compute every mode (default: one of each conjugate pair, the other "
                         "filled by conjugation)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-source-pair", action="store_true",
                    help="skip the generated-versus-stored tensor pair (hash workloads)")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the interaction-factor and derivative-tensor legs")
    ap.add_argument("--profile-steps", type=int, default=2,
                    help="eager steps with an event pair around every kernel (0: none)")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    for leg in ("fp64", "fp32"):
        ap.add_argument(f"--{leg}-steps", type=int, default=None,
                        help=f"timed steps of the {leg.upper()} comparison (default: --steps, "
                             "or 1 for systems above 128 states)")
        ap.add_argument(f"--{leg}-warmup", type=int, default=None,
                        help=f"warmup steps of the {leg.upper()} comparison (default: --warmup, "
                             "or 0 for systems above 128 states)")
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
    conj = not args.no_conj
    log(f"[bench] workload {args.workload}: n={s.n} orders={s.orders} conjugate pairs={conj}")

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
        e = {f"P{M}": err_summary(r["P"][M][modes], refP[M]) for M in s.orders}
        e["npf"] = err_summary(r["npf"][:, modes].T, ref_npf.T)
        return e

    progress = s.n > 128
    profile = 0 if args.no_profile else args.profile_steps
    res = time_path(sysm, s, args.precision, args.steps, args.warmup, device, profile,
                    budget_for(args.workload, args.precision), progress, conj)
    plan = res["plan"]
    entries = plan.modal_entries
    value = entries / (res["ms_per_step"] * 1e-3)
    err = errors(res)
    log(f"[bench] {args.precision}: {res['ms_per_step']:.3f} ms/step, {value:.3e} entries/s, err {err}")

    def leg(prec):
        torch.cuda.empty_cache()
        st, wu = leg_counts(args, s, prec)
        r = time_path(sysm, s, prec, st, wu, device, 0, budget_for(args.workload, prec),
                      progress, conj)
        v = entries / (r["ms_per_step"] * 1e-3)
        e = errors(r)
        log(f"[bench] {prec}: {r['ms_per_step']:.3f} ms/step, {v:.3e} entries/s, err {e}")
        return {"value": v, "ms_per_step": r["ms_per_step"], "rel_err": e,
                "speedup_of_selected": value / v, "steps": st, "warmup": wu,
                "budget_bytes": budget_for(args.workload, prec),
                "block_modes": r["plan"].block_modes, "blocks": r["plan"].n_blocks}

    legs = {p: leg(p) for p in ("fp32", "fp64")
            if p != args.precision and not getattr(args, f"no_{p}")}

    pair = None
    if s.hashed and not args.no_source_pair:
        torch.cuda.empty_cache()
        pair = source_pair(s, sysm, args.precision, conj, device, SOURCE_PAIR_BUDGET, errors)
        log(f"[bench] generated vs stored tensors: "
            f"{pair['generated']['ms_per_step']:.1f} / {pair['stored']['ms_per_step']:.1f} ms")

    inter = taylor = None
    if not args.no_next:
        torch.cuda.empty_cache()
        inter = interaction_leg(s, sysm, args.precision, budget_for(args.workload, args.precision),
                                conj, device, refP, modes)
        log(f"[bench] interaction factors: {inter['ms_per_step']:.3f} ms, err {inter['rel_err']}")
        taylor = taylor_leg(device)
        log(f"[bench] derivative tensors: {taylor}")

    roof = None
    if res["kernels"]:
        psteps = res["profile_steps"]
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
                "traffic_GBps": None,
                "algorithmic_bytes": byts, "algorithmic_flops": flops, "kernel": name,
                "avg_launch_ms": tot / cnt, "launches_per_step": cnt / psteps,
                "share_of_step": tot / psteps / res["ms_per_step"],
                "timing": f"HIP events around every launch on its stream, {psteps} eager "
                          "steps after the timed ones"}
        if roof["traffic"]:
            roof["traffic_GBps"] = roof["traffic"] / avg_s / 1e9
        if mfma:
            roof["executed_mfma_frac"] = achieved * SPLIT_PRODUCTS[args.precision] / peak
        log(f"[bench] kernels: " + ", ".join(f"{k}={v[1] / psteps:.3f}ms"
                                             for k, v in sorted(res['kernels'].items())))

    cpu = None if args.no_cpu_baseline else cpu_baseline(s, entries)

    line = {
        "metric": METRIC, "value": value, "unit": "modal entries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.precision], "data": "synthetic",
        "config": {"workload": args.workload, "n": s.n, "orders": s.orders,
                   "precision": args.precision, "modal_entries_per_step": entries,
                   "conjugate_pairs": conj, "output_modes": plan.output_modes,
                   "computed_modes": plan.computed_modes,
                   "block_modes": plan.block_modes, "blocks": plan.n_blocks,
                   "workspace_bytes": plan.workspace_bytes,
                   "budget_bytes": budget_for(args.workload, args.precision),
                   "oracle_checked_modes": modes},
        "eager_ms_per_step": res.get("eager_ms_per_step"),
        "rel_err_vs_oracle": err,
        "fp64_gpu": legs.get("fp64"),
        "fp32_gpu": legs.get("fp32"),
        "tensor_source_pair": pair,
        "interaction_factors": inter,
        "derivative_tensors": taylor,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
