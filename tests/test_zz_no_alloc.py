"""npf_run_static: the hot path on the library's own static workspace (for callers that
cannot allocate device memory), through the C ABI on the GPU.

Two calls in a row on the same GPU -- the second on a smaller system, so the array keeps
the first call's contents -- each equal bitwise to npf_run with a caller workspace (the
same kernels and launch order), and within the parity bound of the oracle.  A plan whose
workspace exceeds the static size is refused before anything runs.
"""
import numpy as np
import pytest

import oracle
from paper_2509_08968_amd import binding as B
from paper_2509_08968_amd import inputs as I
from tests.helpers import check

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "bf16x3": 1e-6}
STATIC_BYTES = 256 << 20


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    return torch, "cuda:0"


def _run_both(torch, dev, s, precision, conj):
    d = B.upload_system(s, dev)
    n, N = s.n, s.order_max
    plan = B.Plan(n, N, precision, s.eps, s.tau, s.delta, support_max=s.support_max,
                  conj_of=B.conj_pairs(s.lam) if conj else None)
    assert plan.workspace_bytes <= STATIC_BYTES
    ws = plan.workspace(dev)
    st = torch.cuda.Stream()
    Pr = torch.full((N - 1, n, n), complex("nan"), dtype=torch.complex128, device=dev)
    Nr = torch.full((n, n), complex("nan"), dtype=torch.complex128, device=dev)
    Ps, Ns = Pr.clone(), Nr.clone()
    plan.run(d.tensors, d.U, d.V, d.lam, ws, Pr, Nr, st)
    plan.run_static(d.tensors, d.U, d.V, d.lam, Ps, Ns, st)
    torch.cuda.synchronize()
    out = (Ps.cpu().numpy(), Ns.cpu().numpy(), Pr.cpu().numpy(), Nr.cpu().numpy())
    plan.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_static_workspace_matches_npf_run(torch_dev, precision):
    torch, dev = torch_dev
    first = I.block_sparse_system(48, [2, 3], 9401)
    second = I.dense_system(20, [2, 3, 4], 9402)
    for s, conj in ((first, False), (second, True)):
        print(f"[static workspace {precision}] n={s.n} orders {s.orders}", flush=True)
        Ps, Ns, Pr, Nr = _run_both(torch, dev, s, precision, conj)
        assert np.array_equal(Ps, Pr) and np.array_equal(Ns, Nr)
        ref = {M: oracle.sym(s, M)["P"] for M in s.orders}
        for M in s.orders:
            check(Ps[M - 2], ref[M], TOL[precision], f"P_{M}")
        check(Ns.T, oracle.assemble(s, sum(ref.values())).T, TOL[precision], "NPF")


def test_static_workspace_refuses_large_plans(torch_dev):
    torch, dev = torch_dev
    s = I.dense_system(120, [2, 3, 4], 9403)
    plan = B.Plan(s.n, s.order_max, "bf16x3")
    assert plan.workspace_bytes > STATIC_BYTES
    d = B.upload_system(s, dev)
    with pytest.raises(B.NpfError) as e:
        plan.run_static(d.tensors, d.U, d.V, d.lam)
    assert e.value.code == B.NPF_E_UNSUPPORTED and "static workspace" in str(e.value)
    plan.close()
