"""Host-side checks of the library (no GPU): exported symbols, Alg. 1 against the paper's
Tables II/III, and the planner's validation and block sizing."""
import ctypes
import json
import os
import re

import pytest

from paper_2509_08968_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "npf.h")).read()
    declared = set(re.findall(r"\b(npf_[a-z0-9_]+)\s*\(", hdr))
    assert declared == set(B.EXPORTED)
    L = ctypes.CDLL(B.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name


def _golden():
    return json.load(open(os.path.join(ROOT, "tests", "golden", "alg1_tables.json")))


@pytest.mark.parametrize("case", _golden()["cases"], ids=lambda c: f"{c['system']}-o{c['order']}")
def test_alg1_reproduces_tables_ii_iii(case):
    g = _golden()
    r = B.alg1_batches(case["n_dim"], case["n_s"], g["limit_gb"], g["bytes_per_entry"])
    assert r["BC"] == case["BC"]
    assert r["max_batch"] == case["max_batch"]
    if case["batches"] >= 1e8:             # printed with 3 significant digits
        assert abs(r["batches"] - case["batches"]) / case["batches"] < 5e-3
    else:
        assert r["batches"] == case["batches"]
    assert abs(r["batch_gb"] - case["batch_gb"]) < 5e-3
    tot = case["total_gb"]
    assert abs(r["total_gb"] - tot) / tot < (5e-2 if tot >= 1e6 else 5e-5)


def test_alg1_no_batching_when_it_fits():
    r = B.alg1_batches(3, 10, 8.0)
    assert r["batches"] == 1 and r["BC"] == [1, 1, 1]


def test_alg1_rejects_bad_arguments():
    with pytest.raises(ValueError):
        B.alg1_batches(3, 0, 8.0)
    with pytest.raises(ValueError):
        B.alg1_batches(3, 10, 0.0)


def test_plan_counts_and_entries():
    p = B.Plan(64, 3, "fp64")
    assert p.unique_tuples[:4] == [1, 64, 2080, 45760]
    assert p.modal_entries == 64 * (2080 + 45760)
    assert p.n_blocks == 1 and p.block_modes == 64
    assert p.workspace_bytes > 0
    p.close()


@pytest.mark.parametrize("kw,code", [
    (dict(n=0, order_max=2), B.NPF_E_INVALID),
    (dict(n=8, order_max=1), B.NPF_E_INVALID),
    (dict(n=8, order_max=7), B.NPF_E_INVALID),
    (dict(n=8, order_max=2, eps=0.0), B.NPF_E_INVALID),
    (dict(n=8, order_max=2, tau=-1.0), B.NPF_E_INVALID),
    (dict(n=8, order_max=2, budget_bytes=-5), B.NPF_E_INVALID),
    (dict(n=128, order_max=4, budget_bytes=1 << 20), B.NPF_E_BUDGET),
    (dict(n=257, order_max=2), B.NPF_E_UNSUPPORTED),
])
def test_plan_rejects(kw, code):
    with pytest.raises(B.NpfError) as e:
        B.Plan(**kw)
    assert e.value.code == code


def test_plan_budget_shrinks_mode_blocks():
    big = B.Plan(128, 4, "fp32")
    small = B.Plan(128, 4, "fp32", budget_bytes=big.workspace_bytes // 3)
    assert small.n_blocks > 1
    assert small.workspace_bytes <= big.workspace_bytes // 3
    assert small.block_modes * small.n_blocks >= 128
    assert small.block_modes * (small.n_blocks - 1) < 128


def test_plan_explicit_block_size():
    p = B.Plan(40, 2, "fp64", block_modes=16)
    assert p.n_blocks == 3 and p.block_modes == 14


def test_plan_accepts_the_largest_size():
    p = B.Plan(256, 4, "bf16x3")
    assert p.unique_tuples[4] == 259 * 258 * 257 * 256 // 24
    assert p.block_modes * p.n_blocks >= 256
    p.close()
