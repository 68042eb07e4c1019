"""Parity of the HIP path with the CPU FP64 oracle, through the C ABI (needs a GPU).

Tolerances (relative Frobenius error per order and per quantity): 1e-10 for the FP64
path, 1e-6 for the FP32 and split-BF16 paths.
"""
import numpy as np
import pytest

import oracle
from paper_2509_08968_amd import binding as B
from paper_2509_08968_amd import inputs as I
from tests.helpers import HIGH_ORDER_CASES, PARITY_CASES, check

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-6, "bf16x3": 1e-6}


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    return torch, "cuda:0"


def _oracle_all(s):
    ref = {M: oracle.sym(s, M, want_C=True, want_h=True) for M in s.orders}
    npf = oracle.assemble(s, sum(r["P"] for r in ref.values()))
    return ref, npf


@pytest.mark.parametrize("case", sorted(PARITY_CASES))
def test_staged_steps_fp64(torch_dev, case):
    torch, dev = torch_dev
    s = PARITY_CASES[case]()
    print(f"[staged fp64] {case}", flush=True)
    ref, _ = _oracle_all(s)
    d = B.upload_system(s, dev)
    plan = B.Plan(s.n, s.order_max, "fp64", s.eps, s.tau, s.delta)
    ws = plan.workspace(dev)
    for M in s.orders:
        UM = plan.unique_tuples[M]
        C = torch.empty((s.n, UM), dtype=torch.complex128, device=dev)
        plan.modal_contract(M, B.NPF_ALL_BLOCKS, d.tensors[M - 2], d.U, d.V, ws, C)
        torch.cuda.synchronize()
        check(C.cpu().numpy(), ref[M]["C"], TOL["fp64"], "C")
        plan.normal_form(M, B.NPF_ALL_BLOCKS, d.lam, C)
        torch.cuda.synchronize()
        check(C.cpu().numpy(), ref[M]["h"], TOL["fp64"], "h")
        P = torch.zeros((s.n, s.n), dtype=torch.complex128, device=dev)
        plan.assemble(M, B.NPF_ALL_BLOCKS, C, d.U, P)
        torch.cuda.synchronize()
        check(P.cpu().numpy(), ref[M]["P"], TOL["fp64"], "P")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["n12-o3-dense", "n9-o4-dense-odd", "n24-o3-blocksparse",
                                  "n72-o3-dense", "n130-o2-dense"])
def test_staged_steps_mixed(torch_dev, case, precision):
    """The staged entry points on the mixed paths (chain in FP32 or split-BF16, C written in
    FP64; divisor, division and reduction in FP64): C, h and P against the oracle."""
    torch, dev = torch_dev
    s = PARITY_CASES[case]()
    print(f"[staged {precision}] {case}", flush=True)
    ref, _ = _oracle_all(s)
    d = B.upload_system(s, dev)
    plan = B.Plan(s.n, s.order_max, precision, s.eps, s.tau, s.delta,
                  support_max=s.support_max)
    ws = plan.workspace(dev)
    for M in s.orders:
        UM = plan.unique_tuples[M]
        C = torch.empty((s.n, UM), dtype=torch.complex128, device=dev)
        plan.modal_contract(M, B.NPF_ALL_BLOCKS, d.tensors[M - 2], d.U, d.V, ws, C)
        torch.cuda.synchronize()
        check(C.cpu().numpy(), ref[M]["C"], TOL[precision], f"C_{M}")
        plan.normal_form(M, B.NPF_ALL_BLOCKS, d.lam, C)
        torch.cuda.synchronize()
        check(C.cpu().numpy(), ref[M]["h"], TOL[precision], f"h_{M}")
        P = torch.zeros((s.n, s.n), dtype=torch.complex128, device=dev)
        plan.assemble(M, B.NPF_ALL_BLOCKS, C, d.U, P)
        torch.cuda.synchronize()
        check(P.cpu().numpy(), ref[M]["P"], TOL[precision], f"P_{M}")
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("case", sorted(PARITY_CASES))
def test_run_matches_oracle(torch_dev, case, precision):
    s = PARITY_CASES[case]()
    print(f"[run {precision}] {case}", flush=True)
    ref, npf_ref = _oracle_all(s)
    npf, Ps = B.compute(s, precision)
    for M in s.orders:
        check(Ps[M], ref[M]["P"], TOL[precision], f"P_{M}")
    check(npf.T, npf_ref.T, TOL[precision], "NPF")


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_blocks_over_modes_match_single_block(torch_dev, precision):
    s = I.dense_system(40, [2, 3], 3201)
    print(f"[blocks {precision}] n=40", flush=True)
    one, P1 = B.compute(s, precision)
    many, P3 = B.compute(s, precision, block_modes=16)
    for M in s.orders:
        assert np.array_equal(P1[M], P3[M])
    assert np.array_equal(one, many)
    ref, npf_ref = _oracle_all(s)
    check(many.T, npf_ref.T, TOL[precision], "NPF")


def test_run_is_deterministic(torch_dev):
    s = I.block_sparse_system(32, [2, 3], 3301)
    print("[determinism] n=32", flush=True)
    a, Pa = B.compute(s, "fp64")
    b, Pb = B.compute(s, "fp64")
    assert np.array_equal(a, b)
    for M in s.orders:
        assert np.array_equal(Pa[M], Pb[M])


@pytest.mark.parametrize("conj", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_workload_n64_o3_blocksparse_full(torch_dev, precision, conj):
    """The n=64, orders 2-3, block-sparse workload at full size, every mode computed or one
    of each conjugate pair."""
    s = I.workload_sparse64()
    print(f"[n64-o3-blocksparse {precision} conj={conj}]", flush=True)
    ref, npf_ref = _oracle_all(s)
    npf, Ps = B.compute(s, precision, conj=conj)
    for M in s.orders:
        check(Ps[M], ref[M]["P"], TOL[precision], f"P_{M}")
    check(npf.T, npf_ref.T, TOL[precision], "NPF")


def test_linear_limit_on_gpu(torch_dev):
    """A_M = 0: NPF is the linear participation factor delta * Phi o Psi^T exactly."""
    s = I.dense_system(16, [2, 3], 3401, delta=0.5)
    for M in s.orders:
        s.A[M] = np.zeros_like(s.A[M])
    npf, Ps = B.compute(s, "fp64")
    assert all(np.abs(P).max() == 0 for P in Ps.values())
    check(npf.T, (0.5 * s.V * s.U.T).T, 1e-15, "NPF")


def test_graph_replay_matches_eager(torch_dev):
    """npf_run replays a captured graph: every replay, with unrelated eager work and
    synchronisations in between, equals the eager result bitwise; new input values behind
    the same pointers are honoured."""
    torch, dev = torch_dev
    s = I.block_sparse_system(48, [2, 3], 3501)
    print("[graph replay] n=48", flush=True)
    d = B.upload_system(s, dev)
    n, N = s.n, s.order_max
    pe = B.Plan(n, N, "bf16x3", s.eps, s.tau, s.delta, graph=False)
    pg = B.Plan(n, N, "bf16x3", s.eps, s.tau, s.delta, graph=True)
    ws_e, ws_g = pe.workspace(dev), pg.workspace(dev)
    st = torch.cuda.Stream()

    def outs():
        return (torch.empty((N - 1, n, n), dtype=torch.complex128, device=dev),
                torch.empty((n, n), dtype=torch.complex128, device=dev))

    Pe, Ne = outs()
    Pg, Ng = outs()
    pe.run(d.tensors, d.U, d.V, d.lam, ws_e, Pe, Ne, st)
    torch.cuda.synchronize()
    ref_P, ref_N = Pe.clone(), Ne.clone()
    for rep in range(4):
        pg.run(d.tensors, d.U, d.V, d.lam, ws_g, Pg, Ng, st)
        torch.cuda.synchronize()
        assert torch.equal(Pg, ref_P) and torch.equal(Ng, ref_N), rep
        junk = torch.randn(1 << 16, device=dev).sum()      # eager work between replays
        pe.run(d.tensors, d.U, d.V, d.lam, ws_e, Pe, Ne, st)
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
    for t in d.tensors:                                     # new values, same pointers
        t.tensors["values"].mul_(2.0)
    torch.cuda.synchronize()
    pg.run(d.tensors, d.U, d.V, d.lam, ws_g, Pg, Ng, st)
    pe.run(d.tensors, d.U, d.V, d.lam, ws_e, Pe, Ne, st)
    torch.cuda.synchronize()
    assert torch.equal(Pg, Pe) and torch.equal(Ng, Ne)
    assert torch.allclose(Pg, 2.0 * ref_P, rtol=1e-5, atol=0)


# Kept before test_many_plans_share_graph_cache: that test fills the library's graph cache,
# after which new argument sets run eagerly.
@pytest.mark.parametrize("precision", ["fp64"])
@pytest.mark.parametrize("case", sorted(HIGH_ORDER_CASES))
def test_high_orders_graph_replay_matches_eager(torch_dev, case, precision):
    """Five and six orders run concurrently inside the replayed graph (a side stream for
    every order below N, the partial sums chained in order): every replay equals the eager
    run bitwise."""
    torch, dev = torch_dev
    s = HIGH_ORDER_CASES[case]()
    print(f"[graph replay high orders] {case} {precision}", flush=True)
    d = B.upload_system(s, dev)
    n, N = s.n, s.order_max
    pe = B.Plan(n, N, precision, s.eps, s.tau, s.delta, graph=False)
    pg = B.Plan(n, N, precision, s.eps, s.tau, s.delta, graph=True)
    ws_e, ws_g = pe.workspace(dev), pg.workspace(dev)
    st = torch.cuda.Stream()
    Pe = torch.empty((N - 1, n, n), dtype=torch.complex128, device=dev)
    Ne = torch.empty((n, n), dtype=torch.complex128, device=dev)
    Pg, Ng = torch.empty_like(Pe), torch.empty_like(Ne)
    pe.run(d.tensors, d.U, d.V, d.lam, ws_e, Pe, Ne, st)
    torch.cuda.synchronize()
    for rep in range(3):
        pg.run(d.tensors, d.U, d.V, d.lam, ws_g, Pg, Ng, st)
        torch.cuda.synchronize()
        assert torch.equal(Pg, Pe) and torch.equal(Ng, Ne), rep
    pg.close()
    pe.close()


def test_many_plans_share_graph_cache(torch_dev):
    """More concurrent-order plans than npf_run keeps graphs for, one after another: each
    runs (captured and replayed while the cache has room, eagerly after that), is checked
    bitwise against an eager run and is destroyed right after its last (still running)
    replay was enqueued.  The graphs outlive their plans; the side streams and events they
    were captured from belong to the library."""
    torch, dev = torch_dev
    st = torch.cuda.Stream()
    for q in range(20):
        n = 20 + 2 * q
        s = I.block_sparse_system(n, [2, 3], 3600 + q)
        print(f"[many plans] q={q} n={n}", flush=True)
        d = B.upload_system(s, dev)
        pe = B.Plan(n, 3, "bf16x3", s.eps, s.tau, s.delta, graph=False)
        pg = B.Plan(n, 3, "bf16x3", s.eps, s.tau, s.delta, graph=True)
        ws_e, ws_g = pe.workspace(dev), pg.workspace(dev)
        Pe = torch.empty((2, n, n), dtype=torch.complex128, device=dev)
        Ne = torch.empty((n, n), dtype=torch.complex128, device=dev)
        Pg, Ng = torch.empty_like(Pe), torch.empty_like(Ne)
        pe.run(d.tensors, d.U, d.V, d.lam, ws_e, Pe, Ne, st)
        for _ in range(2):
            pg.run(d.tensors, d.U, d.V, d.lam, ws_g, Pg, Ng, st)
        pg.close()                    # its replay may still be running
        torch.cuda.synchronize()
        assert torch.equal(Pg, Pe) and torch.equal(Ng, Ne), q
        pe.close()


@pytest.fixture(scope="module")
def dense128():
    """n=128, orders 2-4 dense with planted resonances and the oracle's P rows for two
    sampled output modes (one of them the mode closest to an order-2 resonance)."""
    s = I.workload_dense128()
    lam = s.lam
    d2 = np.abs(lam[None, :, None] + lam[None, None, :] - lam[:, None, None]).reshape(s.n, -1).min(1)
    modes = [int(np.argmin(d2)), 5]
    ref = {M: oracle.sym(s, M, modes=modes)["P"] for M in s.orders}
    return s, modes, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["bf16x3", "fp32", "fp64"])
def test_workload_n128_o4_dense_sampled(torch_dev, dense128, precision):
    """n=128, orders 2-4, dense, under a 64 GiB workspace budget, one mode of each
    conjugate pair computed (the benchmark's configuration).  P_M rows and NPF columns of
    the sampled modes are compared with the oracle, each mode on its own: each mode's chain
    is independent, so these are exact checks of the full-size run (mode 5 is filled by
    conjugation from mode 4)."""
    torch, dev = torch_dev
    s, modes, ref = dense128
    print(f"[n128-o4 {precision}] modes {modes}", flush=True)
    npf, Ps = B.compute(s, precision, budget_bytes=64 << 30, conj=True)
    for M in s.orders:
        check(Ps[M][modes], ref[M], TOL[precision], f"P_{M}")
    z = np.stack([s.delta * s.U[i, :] for i in modes])          # [modes, states]
    npf_cols = s.V[:, modes] * (z + sum(ref.values())).T
    check(npf[:, modes].T, npf_cols.T, TOL[precision], "NPF")


# Orders 5 and 6 run in FP64 only (the mixed paths refuse them: their FP32 C, shared by
# every ordering of a sorted tuple, misses 1e-6 there; a host test checks the refusal).
@pytest.mark.parametrize("case", sorted(HIGH_ORDER_CASES))
def test_high_orders_match_oracle(torch_dev, case):
    torch, dev = torch_dev
    s = HIGH_ORDER_CASES[case]()
    print(f"[high orders fp64] {case}", flush=True)
    ref, npf_ref = _oracle_all(s)
    npf, Ps = B.compute(s, "fp64", dev)
    for M in s.orders:
        check(Ps[M], ref[M]["P"], TOL["fp64"], f"P_{M}")
    check(npf.T, npf_ref.T, TOL["fp64"], "NPF")


@pytest.mark.parametrize("case", sorted(HIGH_ORDER_CASES))
def test_high_orders_staged_steps_fp64(torch_dev, case):
    torch, dev = torch_dev
    s = HIGH_ORDER_CASES[case]()
    print(f"[high orders staged fp64] {case}", flush=True)
    ref, _ = _oracle_all(s)
    d = B.upload_system(s, dev)
    plan = B.Plan(s.n, s.order_max, "fp64", s.eps, s.tau, s.delta)
    ws = plan.workspace(dev)
    for M in s.orders:
        C = torch.empty((s.n, plan.unique_tuples[M]), dtype=torch.complex128, device=dev)
        plan.modal_contract(M, B.NPF_ALL_BLOCKS, d.tensors[M - 2], d.U, d.V, ws, C)
        torch.cuda.synchronize()
        check(C.cpu().numpy(), ref[M]["C"], TOL["fp64"], f"C_{M}")
        plan.normal_form(M, B.NPF_ALL_BLOCKS, d.lam, C)
        P = torch.zeros((s.n, s.n), dtype=torch.complex128, device=dev)
        plan.assemble(M, B.NPF_ALL_BLOCKS, C, d.U, P)
        torch.cuda.synchronize()
        check(P.cpu().numpy(), ref[M]["P"], TOL["fp64"], f"P_{M}")
    plan.close()


def _zero_order3():
    s = I.block_sparse_system(24, [2, 3], 3111)
    s.A[3] = np.zeros_like(s.A[3])          # sent sparse: no columns at all
    return s


EMPTY_CASES = {
    "n24-o3-zero-tensor": _zero_order3,
    "n10-o2o4-missing-o3": lambda: I.dense_system(10, [2, 4], 3112),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("case", sorted(EMPTY_CASES))
def test_empty_tensor_gives_zero_order(torch_dev, case, precision):
    """A derivative tensor with no entries (an all-zero tensor sent sparse, or an order the
    system does not have) contributes exactly nothing: P_3 is zero bit for bit, the other
    orders and the NPF match the oracle.  The upper index goes first on every order."""
    s = EMPTY_CASES[case]()
    print(f"[empty tensor] {case} {precision}", flush=True)
    ref = {M: oracle.sym(s, M) for M in s.orders}
    npf_ref = oracle.assemble(s, sum(r["P"] for r in ref.values()))
    npf, Ps = B.compute(s, precision, support_max=0)
    assert not np.any(Ps[3]), "P_3 must be exactly zero"
    for M in s.orders:
        if M != 3:
            check(Ps[M], ref[M]["P"], TOL[precision], f"P_{M}")
    check(npf.T, npf_ref.T, TOL[precision], "NPF")


# ------------------------------------------------------------------ the clamp of Alg. 2 step 9
CLAMP_CASES = {
    "n28-o3": lambda: I.clamp_system(28, [2, 3], 9128),        # operands resident (n <= 64)
    "n40-o4": lambda: I.clamp_system(40, [2, 3, 4], 9140),
    "n80-o3": lambda: I.clamp_system(80, [2, 3], 9180),        # t-range kernels (n > 64)
    "n100-o4": lambda: I.clamp_system(100, [2, 3, 4], 9200),
}


def clamp_modes(s):
    """Output modes with a divisor of modulus below 2 eps (orders 2 and 3 from the sums,
    order 4 from exact matches of pair sums, which the dyadic spectrum makes exact), plus
    the first and last mode; every mode for small systems."""
    if s.n <= 40:
        return list(range(s.n))
    lam = s.lam
    hit = {0, s.n - 1}
    for M in (2, 3):
        if M in s.orders:
            t = I.sorted_tuples(s.n, M)
            d = np.abs(lam[t].sum(1)[None, :] - lam[:, None]).min(1)
            hit |= set(np.nonzero(d < 2 * s.eps)[0].tolist())
    if 4 in s.orders:
        t = I.sorted_tuples(s.n, 2)
        sums = set(lam[t].sum(1).tolist())
        for j in range(s.n):
            if any((lam[j] - x) in sums for x in sums):
                hit.add(j)
    return sorted(hit)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("case", sorted(CLAMP_CASES))
def test_clamp_matches_oracle(torch_dev, case, precision):
    """Divisors exactly 0, just below eps (clamped to eps) and just above it (kept), exact in
    FP64 on both sides: P rows and NPF columns of the affected modes against the oracle."""
    s = CLAMP_CASES[case]()
    modes = clamp_modes(s)
    print(f"[clamp {precision}] {case} modes {modes if len(modes) < 12 else len(modes)}", flush=True)
    ref = {M: oracle.sym(s, M, modes=modes)["P"] for M in s.orders}
    npf, Ps = B.compute(s, precision)
    for M in s.orders:
        check(Ps[M][modes], ref[M], TOL[precision], f"P_{M}")
    z = np.stack([s.delta * s.U[i, :] for i in modes])
    check(npf[:, modes].T, s.V[:, modes].T * (z + sum(ref.values())), TOL[precision], "NPF")


def test_clamp_staged_fp64_elementwise(torch_dev):
    """Staged FP64 path on a clamp system: C and h element by element against the oracle,
    and h = C / eps exactly where the oracle clamps."""
    torch, dev = torch_dev
    s = CLAMP_CASES["n40-o4"]()
    print("[clamp staged fp64] n40-o4", flush=True)
    d = B.upload_system(s, dev)
    plan = B.Plan(s.n, s.order_max, "fp64", s.eps, s.tau, s.delta)
    ws = plan.workspace(dev)
    clamped = 0
    for M in s.orders:
        ref = oracle.sym(s, M, want_C=True, want_h=True)
        C = torch.empty((s.n, plan.unique_tuples[M]), dtype=torch.complex128, device=dev)
        plan.modal_contract(M, B.NPF_ALL_BLOCKS, d.tensors[M - 2], d.U, d.V, ws, C)
        torch.cuda.synchronize()
        Cg = C.cpu().numpy()
        plan.normal_form(M, B.NPF_ALL_BLOCKS, d.lam, C)
        torch.cuda.synchronize()
        hg = C.cpu().numpy()
        mask = (ref["h"] == ref["C"] / s.eps) & (ref["C"] != 0)
        clamped += int(mask.sum())
        scale = np.abs(ref["h"]).max(axis=1, keepdims=True)
        assert np.all(np.abs(hg - ref["h"]) <= 1e-10 * scale), M
        assert np.all(np.abs(hg[mask] - Cg[mask] / s.eps) <= 1e-12 * np.abs(hg[mask])), M
    assert clamped >= 10, clamped
    plan.close()
