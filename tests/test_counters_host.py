"""The counter summaries that bench.py reports as roofline.traffic (host only).

Synthetic rocprofv3 counter files stand in for two passes over one batched step: every
shared launch gets a distinct byte count, so the summary must attribute each to its launch
name, scale it by the copy probe, and refuse a dispatch whose kernel does not match the
name it would be given.
"""
import csv

import pytest

import bench_counters as C

W = "batch256-o3-blocksparse"


def _symbol(name):
    npad, order, kind = name.split("_")[1][2:], name.split("_")[2][1:], name.split("_")[3]
    kern = "fused_bf3_tr_multi" if kind == "fused" else "stage_bf3_tr_multi"
    if int(npad) <= 64:
        kern = kern.replace("_tr", "")
    return f"void npf::(anonymous namespace)::{kern}<{npad}, {order}, 2>(npf::Bf3Args const*)"


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Value"])
        w.writeheader()
        for i, (k, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Value": v})


@pytest.fixture(scope="module")
def names():
    return C.batch_launch_names(W)


def _passes(tmp_path, names, swap=False):
    # copy probe of 256 MiB that the counter reports as 128 MiB (factor 2), then one step:
    # a per-system launch between every shared launch, and the shared launches.
    rows = [("__amd_rocclr_copyBuffer", 128 * 1024.0)]
    order = list(names)
    if swap:
        order[0], order[-1] = order[-1], order[0]
    for q, nm in enumerate(order):
        rows.append(("npf::(anonymous namespace)::prepare(...)", 1.0))
        rows.append((_symbol(nm), float(names.index(nm) + 1)))
    f, w = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _write(f, rows)
    _write(w, rows)
    return str(f), str(w)


def test_batch_launches_are_named_in_dispatch_order(tmp_path, names):
    assert len(names) == len(set(names)) == 36
    f, w = _passes(tmp_path, names)
    t = C.traffic(W, "bf16x3", f, w, 256)
    assert set(t) == set(names)
    for i, nm in enumerate(names):
        # KiB counter value (i + 1), times the copy factor 2, in bytes
        assert t[nm]["fetch_bytes_per_launch"] == pytest.approx((i + 1) * 2 * 1024)
        assert t[nm]["launches_per_step"] == 1


def test_mismatched_dispatch_is_refused(tmp_path, names):
    f, w = _passes(tmp_path, names, swap=True)
    with pytest.raises(ValueError):
        C.traffic(W, "bf16x3", f, w, 256)
