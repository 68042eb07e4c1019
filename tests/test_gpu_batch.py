"""Batched operating points (npf_batch_*) on the GPU through the C ABI.

Systems of uneven n share each chain-stage and fused-stage launch; every system's P_M and
NPF must match the oracle (split-BF16 tolerance) and the single-system path, in one wave
or several under a workspace budget, eagerly and as a replayed graph, before and after the
autotuner changes the workgroup counts.
"""
import numpy as np
import pytest

import oracle
from paper_2509_08968_amd import binding as B
from paper_2509_08968_amd import inputs as I
from tests.helpers import check

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    return torch, "cuda:0"


def mixed_systems():
    """Every padded size class (32 .. 160), orders 2-3 and one order-4 system, sparse and
    dense tensors, even and odd n."""
    ss = [I.block_sparse_system(n, [2, 3], 7000 + n) for n in (10, 32, 40, 64, 70, 96, 100, 130, 160)]
    ss.append(I.dense_system(20, [2, 3, 4], 7100))
    ss.append(I.dense_system(37, [2], 7101))
    return ss


@pytest.fixture(scope="module")
def mixed_reference():
    ss = mixed_systems()
    ref = []
    for s in ss:
        modes = list(range(s.n)) if s.n <= 40 else sorted({0, s.n // 2 + 1, s.n - 1})
        P = {M: oracle.sym(s, M, modes=modes)["P"] for M in s.orders}
        z = np.stack([s.delta * s.U[i, :] for i in modes])
        ref.append((modes, P, s.V[:, modes] * (z + sum(P.values())).T))
    return ss, ref


def check_against(results, ss, ref):
    for q, (s, (npf, Ps)) in enumerate(zip(ss, results)):
        modes, P, cols = ref[q]
        for M in s.orders:
            check(Ps[M][modes], P[M], TOL, f"system {q} n={s.n} P_{M}")
        check(npf[:, modes].T, cols.T, TOL, f"system {q} n={s.n} NPF")


@pytest.mark.parametrize("budget", [0, 6 << 30])
def test_batch_matches_oracle_and_single_runs(torch_dev, mixed_reference, budget):
    ss, ref = mixed_reference
    print(f"[batch] {len(ss)} systems, budget {budget}", flush=True)
    res = B.compute_batch(ss, budget_bytes=budget)
    check_against(res, ss, ref)
    for s, (npf, Ps) in zip(ss, res):
        one, P1 = B.compute(s, "bf16x3")
        for M in s.orders:
            check(Ps[M], P1[M], 1e-12, f"n={s.n} P_{M} vs single")
        check(npf.T, one.T, 1e-12, f"n={s.n} NPF vs single")


def test_batch_graph_replay_and_autotuner(torch_dev, mixed_reference):
    torch, dev = torch_dev
    ss, ref = mixed_reference
    print("[batch graph/tune]", flush=True)
    devs = [B.upload_system(s, dev) for s in ss]
    b = B.Batch(ss, budget_bytes=6 << 30)
    ws = b.workspace(dev)
    mk = lambda: ([torch.empty((s.order_max - 1, s.n, s.n), dtype=torch.complex128, device=dev)
                   for s in ss], [torch.empty((s.n, s.n), dtype=torch.complex128, device=dev) for s in ss])
    Pe, Ne = mk()
    b.run(devs, ws, Pe, Ne, torch.cuda.default_stream())        # NULL stream: eager
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    Pg, Ng = mk()
    for rep in range(3):
        b.run(devs, ws, Pg, Ng, st)                              # captured, then replayed
        torch.cuda.synchronize()
        for q in range(len(ss)):
            assert torch.equal(Pg[q], Pe[q]) and torch.equal(Ng[q], Ne[q]), (rep, q)
        float(torch.randn(1 << 16, device=dev).sum())            # eager work in between
    chosen = b.tune(devs, ws, Pe, Ne, st)
    assert len(chosen) == b.report["shared_launches"]
    assert all(c in (256, 512, 1024, 2048, 4096) for c in chosen)
    b.run(devs, ws, Pg, Ng, st)
    torch.cuda.synchronize()
    res = [(Ng[q].cpu().numpy(), {M: Pg[q][M - 2].cpu().numpy() for M in s.orders})
           for q, s in enumerate(ss)]
    check_against(res, ss, ref)
    b.close()


@pytest.mark.timeout(900)
def test_workload_batch256_sampled(torch_dev):
    """256 block-sparse systems, n uniform over even values in [32, 160], orders 2-3, under a
    128 GiB workspace budget: sampled systems and modes against the oracle."""
    ss = I.workload_batch()
    print("[batch256]", flush=True)
    res = B.compute_batch(ss, budget_bytes=128 << 30)
    order = np.argsort([s.n for s in ss], kind="stable")
    rng = np.random.default_rng(I.BASE_SEED + 3 + 1000)
    picks = sorted({int(order[0]), int(order[-1]), *[int(x) for x in rng.choice(len(ss), 3, replace=False)]})
    for q in picks:
        s = ss[q]
        modes = sorted({0, s.n // 2 + 1, s.n - 1})
        P = {M: oracle.sym(s, M, modes=modes)["P"] for M in s.orders}
        npf, Ps = res[q]
        for M in s.orders:
            check(Ps[M][modes], P[M], TOL, f"system {q} n={s.n} P_{M}")
        z = np.stack([s.delta * s.U[i, :] for i in modes])
        check(npf[:, modes].T, s.V[:, modes].T * (z + sum(P.values())), TOL, f"system {q} NPF")


def test_batch_more_argument_sets_than_cached_graphs(torch_dev):
    """Six argument sets (distinct output buffers) through one batch: the first four are
    captured and replayed, the rest run eagerly, no cached graph is destroyed while the
    batch lives, and every run equals the eager result bitwise.  The batch is then destroyed
    right after enqueueing a replay (its graphs are released once that launch is done)."""
    torch, dev = torch_dev
    ss = [I.block_sparse_system(n, [2, 3], 7200 + n) for n in (24, 40, 70)]
    print("[batch argument sets] 3 systems, 6 sets", flush=True)
    devs = [B.upload_system(s, dev) for s in ss]
    b = B.Batch(ss)
    ws = b.workspace(dev)
    mk = lambda: ([torch.empty((s.order_max - 1, s.n, s.n), dtype=torch.complex128, device=dev)
                   for s in ss], [torch.empty((s.n, s.n), dtype=torch.complex128, device=dev) for s in ss])
    Pe, Ne = mk()
    b.run(devs, ws, Pe, Ne, torch.cuda.default_stream())        # NULL stream: eager
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    sets = [mk() for _ in range(6)]
    for rep in range(2):
        for k, (Pg, Ng) in enumerate(sets):
            b.run(devs, ws, Pg, Ng, st)
            torch.cuda.synchronize()
            for q in range(len(ss)):
                assert torch.equal(Pg[q], Pe[q]) and torch.equal(Ng[q], Ne[q]), (rep, k, q)
    b.run(devs, ws, sets[0][0], sets[0][1], st)                  # a replay still in flight
    b.close()
    torch.cuda.synchronize()
    for q in range(len(ss)):
        assert torch.equal(sets[0][0][q], Pe[q]) and torch.equal(sets[0][1][q], Ne[q]), q
