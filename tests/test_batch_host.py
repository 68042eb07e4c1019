"""Host-side checks of the batched-systems planner (no GPU): waves under a budget,
shared launches per padded size, entry counts and argument errors."""
import math

import pytest

from paper_2509_08968_amd import binding as B
from paper_2509_08968_amd import inputs as I


def systems():
    return [I.block_sparse_system(n, [2, 3], 7000 + n) for n in (10, 40, 70, 130)] + \
        [I.dense_system(20, [2, 3, 4], 7100)]


def test_entries_and_single_wave():
    ss = systems()
    b = B.Batch(ss)
    r = b.report
    assert r["systems"] == len(ss) and r["waves"] == 1
    assert r["modal_entries"] == sum(s.n * math.comb(s.n + M - 1, M) for s in ss for M in s.orders)
    # one shared fused launch per (padded size, order); chain stages only for systems that
    # do not take the lower-indices-first route (sparse with a support bound, orders <= 3)
    want = set()
    for s in ss:
        np_ = (s.n + 31) // 32 * 32
        for M in s.orders:
            want.add((np_, M, M))
            if not (s.support_max and ((M == 3 and s.n > 64) or (M == 2 and s.n > 96))):
                want.update((np_, M, i) for i in range(1, M))
    assert r["shared_launches"] == len(want)


def test_budget_makes_waves():
    ss = systems()
    one = B.Batch(ss).report
    biggest = max(B.Plan(s.n, s.order_max, "bf16x3", support_max=s.support_max).workspace_bytes
                  for s in ss)
    b = B.Batch(ss, budget_bytes=biggest + (1 << 20))
    assert b.report["waves"] >= 2
    assert b.report["workspace_bytes"] <= one["workspace_bytes"]


def test_budget_below_one_system_is_an_error():
    with pytest.raises(B.NpfError) as e:
        B.Batch(systems(), budget_bytes=1 << 20)
    assert e.value.code == 2


def test_unsupported_requests():
    s = I.dense_system(12, [2, 3, 4, 5], 7200)
    with pytest.raises(B.NpfError) as e:
        B.Batch([s])
    assert e.value.code == 4
