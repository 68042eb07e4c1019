"""Summaries of rocprofv3 output for the benchmark workloads (host only, no GPU).

Turns the CSV files of `rocprofv3 --kernel-trace --stats` and of two `rocprofv3 --pmc`
passes (FETCH_SIZE, then WRITE_SIZE) into short text summaries and a JSON file with the
HBM bytes per launch of every kernel of one step, which bench.py reports as
roofline.traffic while the kernel sources are unchanged.

Counter scaling: bench.py --copy-probe-mib X runs one device copy of X MiB before the
workload; the factor that maps that copy's FETCH_SIZE (resp. WRITE_SIZE) to X MiB is
applied to every dispatch.  Dispatches are named by the launch order of npf_run, which is
fixed for a plan: prepare; per order M: the per-row tables (when the lower indices go
first); per mode block: the upper-index contraction (two launches for sparse tensors: clear +
scatter) and stages 1..M-1, or the per-row Psi step; the fused last stage; one partial-sum
launch (which also writes the NPF for the last order).

usage: python bench_counters.py trace WORKLOAD PRECISION STATS_CSV OUT_DIR CMD
       python bench_counters.py sq WORKLOAD PRECISION COUNTER_CSV OUT_DIR CMD
       python bench_counters.py traffic WORKLOAD PRECISION FETCH_CSV WRITE_CSV
           COPY_MIB OUT_DIR CMD...
"""
from __future__ import annotations

import csv
import functools
import json
import os
import sys
from collections import defaultdict


def launch_names(workload: str, precision: str, budget: int = 0, conj: bool = True):
    """Kernel names of one npf_run step, in dispatch order, for the plan bench.py makes
    (one mode of each conjugate pair computed unless ``conj`` is False)."""
    from paper_2509_08968_amd import binding as B
    from paper_2509_08968_amd import inputs as I
    s = I.WORKLOADS[workload]()
    plan = B.Plan(s.n, s.order_max, precision, s.eps, s.tau, s.delta, budget_bytes=budget,
                  support_max=s.support_max, conj_of=B.conj_pairs(s.lam) if conj else None)
    # Graph replays of single-block plans with several orders run the orders concurrently;
    # their dispatch order is the capture order: every order's launches, highest order first,
    # then the partial sums of every order in ascending order (the workloads here fit the
    # per-order workspace of that mode).
    concurrent = plan.n_blocks == 1 and s.order_max >= 3
    names = ["prepare"]
    reduces = []
    orders = range(s.order_max, 1, -1) if concurrent else range(2, s.order_max + 1)
    for M in orders:
        sparse = s.support.get(M) is not None and M not in s.hashed
        tucker = sparse and 1 <= s.support_max <= 8 and (
            (M == 3 and (s.n > 64 or precision == "fp64")) or (M == 2 and s.n > 96))
        if tucker:
            names += [f"o{M}_tucker_support.rows", f"o{M}_tucker_support.inverse"]
            names += ([f"o{M}_tucker_w.y", f"o{M}_tucker_w"] if M == 3 else [f"o{M}_tucker_w"])
        for _ in range(plan.n_blocks):
            if tucker:
                names.append(f"o{M}_tucker_psi")
            elif sparse:
                names += [f"o{M}_psi_a.clear", f"o{M}_psi_a"]
            else:
                names.append(f"o{M}_psi_a")
            if not tucker:
                names += [f"o{M}_stage{i}" for i in range(1, M)]
            names.append(f"o{M}_fused")
            (reduces if concurrent else names).append(f"o{M}_reduce")
    plan.close()
    return names + sorted(reduces)


@functools.lru_cache(maxsize=None)
def batch_launch_names(workload: str):
    """Names of the shared (multi-system) launches of one batched step, in dispatch order,
    as bench.py names them: w<wave>_np<padded n>_o<order>_stage<i> | _fused.  Every chain
    stage and last stage of a batch runs in one of these launches (the kernels whose names end
    in _multi); the per-system launches around them are not named here.  The launch records
    are listed by wave, padded size, order and stage; a run launches them by wave, order and
    stage (the fused last stage after stage M-1), each over the padded sizes in turn."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import bench
    from paper_2509_08968_amd import binding as B
    from paper_2509_08968_amd import inputs as I
    if workload != bench.BATCH_WORKLOAD:
        raise ValueError(f"not a batched workload: {workload}")
    b = B.Batch(I.workload_batch(), bench.BATCH_BUDGET)
    recs = b.launches()
    b.close()
    order = sorted(range(len(recs)), key=lambda q: (
        recs[q]["wave"], recs[q]["order"],
        recs[q]["stage"] if recs[q]["kind"] == 0 else recs[q]["order"], q))
    return tuple(f"w{recs[q]['wave']}_np{recs[q]['npad']}_o{recs[q]['order']}_" +
                 (f"stage{recs[q]['stage']}" if recs[q]["kind"] == 0 else "fused") for q in order)


def _dispatches(path):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in rows]


def _scale(disp, copy_mib):
    copies = [v for k, v in disp if k.startswith("__amd_rocclr_copyBuffer")]
    big = max(copies)
    return (copy_mib * 1024.0) / big            # counters are in KiB


def traffic(workload, precision, fetch_csv, write_csv, copy_mib, budget=0):
    batched = workload.startswith("batch")
    names = batch_launch_names(workload) if batched else launch_names(workload, precision, budget)
    out = {}
    for ctr, path in (("fetch", fetch_csv), ("write", write_csv)):
        disp = _dispatches(path)
        f = _scale(disp, copy_mib)
        lib = [(k, v) for k, v in disp if "npf::" in k and (not batched or "_multi" in k)]
        steps = len(lib) // len(names)
        acc = defaultdict(list)
        for s in range(steps):
            for i, nm in enumerate(names):
                k, v = lib[s * len(names) + i]
                if batched:
                    # the symbol must be the named kind of kernel at the named padded size
                    kind = "fused" if nm.endswith("fused") else "stage"
                    npad = nm.split("_")[1][2:]
                    if kind not in k or f"<{npad}," not in k:
                        raise ValueError(f"dispatch {k[:80]} does not match launch {nm}")
                acc[nm].append((k, v * f * 1024.0))
        for nm, vals in acc.items():
            d = out.setdefault(nm, {"symbol": vals[0][0][:100]})
            blocks = names.count(nm)
            d[f"{ctr}_bytes_per_launch"] = sum(v for _, v in vals) / len(vals)
            d[f"{ctr}_scale"] = f
            d["launches_per_step"] = blocks
    for d in out.values():
        d["bytes_per_launch"] = d.get("fetch_bytes_per_launch", 0.0) + d.get("write_bytes_per_launch", 0.0)
    return out


def write_trace(workload, precision, stats_csv, out_dir, cmd):
    """Kernel-trace statistics summary (profiles/kernel_trace_<workload>_<precision>.txt)."""
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# rocprofv3 kernel-trace statistics, {workload}, {precision}",
             "# command (repo root, TMPDIR=/tmp):", f"#   {cmd}",
             "# calls  total_ms  avg_us  min_us  max_us  pct  kernel"]
    for r in rows:
        lines.append(f"{int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:10.2f} "
                     f"{float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):6.2f}  {r['Name'][:100]}")
    with open(os.path.join(out_dir, f"kernel_trace_{workload}_{precision}.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


def write_traffic(workload, precision, fetch_csv, write_csv, copy_mib, out_dir, cmds):
    """HBM traffic summary and the per-launch JSON that bench.py reads."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import bench
    budget = bench.budget_for(workload, precision)
    t = traffic(workload, precision, fetch_csv, write_csv, float(copy_mib), budget)
    js = {"workload": workload, "precision": precision,
          "source_digest": bench.kernel_source_digest(), "kernels": t,
          "note": "HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled "
                  "by the ratio of a device copy of known size to what the counter reports "
                  "for it; valid for the kernel sources with this digest"}
    with open(os.path.join(out_dir, f"traffic_{workload}_{precision}.json"), "w") as f:
        json.dump(js, f, indent=1)
    first = next(iter(t.values()))
    lines = [f"# HBM traffic per launch, {workload}, {precision}",
             "# commands (repo root, TMPDIR=/tmp):", *[f"#   {c}" for c in cmds],
             f"# counter scale factors (copy of {copy_mib} MiB): fetch "
             f"{first['fetch_scale']:.3f}, write {first['write_scale']:.3f}",
             "# kernel  launches/step  fetch_GB  write_GB  symbol"]
    for nm, d in sorted(t.items(), key=lambda kv: -kv[1]["bytes_per_launch"]):
        lines.append(f"{nm:24s} {d['launches_per_step']:3d} {d['fetch_bytes_per_launch'] / 1e9:10.4f} "
                     f"{d['write_bytes_per_launch'] / 1e9:10.4f}  {d['symbol']}")
    with open(os.path.join(out_dir, f"hbm_traffic_{workload}_{precision}.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


SQ_COUNTERS = ("SQ_WAVE_CYCLES", "SQ_BUSY_CU_CYCLES", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_INSTS_VALU",
               "SQ_INSTS_MFMA", "SQ_INSTS_LDS", "SQ_WAIT_INST_ANY", "SQ_LDS_BANK_CONFLICT")


def write_sq(workload, precision, csv_path, out_dir, cmd, budget=0):
    """Instruction-mix summary of one rocprofv3 --pmc pass over SQ_COUNTERS
    (profiles/sq_mix_<workload>_<precision>.txt): per launch of each kernel of a step, the
    ratios that do not depend on how the counters are normalised over SIMDs and XCDs."""
    names = launch_names(workload, precision, budget)
    per = defaultdict(dict)                      # dispatch id -> {counter: value}
    kern = {}
    for r in csv.DictReader(open(csv_path)):
        d = int(r["Dispatch_Id"])
        per[d][r["Counter_Name"]] = per[d].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        kern[d] = r["Kernel_Name"]
    lib = [d for d in sorted(per) if "npf::" in kern[d]]
    steps = len(lib) // len(names)
    acc = defaultdict(lambda: defaultdict(float))
    for s in range(steps):
        for i, nm in enumerate(names):
            for c, v in per[lib[s * len(names) + i]].items():
                acc[nm][c] += v
    lines = [f"# SQ instruction mix per kernel, {workload}, {precision}",
             "# command (repo root, TMPDIR=/tmp):", f"#   {cmd}",
             "# valu/mfma, lds/mfma: instructions issued per MFMA instruction; mfma_busy/cu_busy:",
             "#   SQ_VALU_MFMA_BUSY_CYCLES / SQ_BUSY_CU_CYCLES (both summed by the counter block);",
             "#   wait/wave: SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES; conflicts/lds: bank-conflict cycles",
             "#   per LDS instruction",
             "# kernel  valu/mfma  lds/mfma  mfma_busy/cu_busy  wait/wave  conflicts/lds  mfma_insts"]
    for nm in dict.fromkeys(names):
        a = acc[nm]
        mf = a.get("SQ_INSTS_MFMA", 0.0)
        q = lambda x, y: (a.get(x, 0.0) / a[y]) if a.get(y) else float("nan")
        lines.append(f"{nm:22s} {q('SQ_INSTS_VALU', 'SQ_INSTS_MFMA'):9.2f} "
                     f"{q('SQ_INSTS_LDS', 'SQ_INSTS_MFMA'):9.2f} "
                     f"{q('SQ_VALU_MFMA_BUSY_CYCLES', 'SQ_BUSY_CU_CYCLES'):9.3f} "
                     f"{q('SQ_WAIT_INST_ANY', 'SQ_WAVE_CYCLES'):9.3f} "
                     f"{q('SQ_LDS_BANK_CONFLICT', 'SQ_INSTS_LDS'):9.3f} {mf / max(steps, 1):12.4g}")
    with open(os.path.join(out_dir, f"sq_mix_{workload}_{precision}.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


def main(argv):
    mode = argv[0]
    if mode == "trace":
        workload, precision, stats_csv, out_dir, cmd = argv[1:6]
        write_trace(workload, precision, stats_csv, out_dir, cmd)
    elif mode == "traffic":
        workload, precision, fetch_csv, write_csv, copy_mib, out_dir = argv[1:7]
        write_traffic(workload, precision, fetch_csv, write_csv, copy_mib, out_dir, argv[7:])
    elif mode == "sq":
        workload, precision, csv_path, out_dir, cmd = argv[1:6]
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        import bench
        write_sq(workload, precision, csv_path, out_dir, cmd, bench.budget_for(workload, precision))
    else:
        raise SystemExit("usage: bench_counters.py trace|traffic|sq ...")


if __name__ == "__main__":
    main(sys.argv[1:])
