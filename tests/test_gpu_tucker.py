"""The lower-indices-first route for sparse tensors (rows involving few states) on the GPU.

The route is taken for order 3 when n > 64 or in FP64, and for order 2 when n > 96; the
cases below cover both sides of each threshold.

With a declared per-row support bound, each row k of a sparse A_M is contracted over its
own states first and Psi is applied after (Alg. 2 steps 2-3 then step 4); without the
bound the same tensors go through the upper-index-first chain.  Both must match the
oracle, each other, and a bound that is too small must make the results NaN.
"""
import numpy as np
import pytest

import oracle
from paper_2509_08968_amd import binding as B
from paper_2509_08968_amd import inputs as I
from tests.helpers import check

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-6, "bf16x3": 1e-6}


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    return torch, "cuda:0"


CASES = {
    "n24-o3": lambda: I.block_sparse_system(24, [2, 3], 8101),
    "n110-o2-ragged": lambda: I.block_sparse_system(110, [2], 8102),    # last block of 2 states
    "n64-o3": I.workload_sparse64,
    "n100-o3": lambda: I.block_sparse_system(100, [2, 3], 8103),
    "n150-o3-blocks32": lambda: I.block_sparse_system(150, [2, 3], 8104),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_rows_first_matches_oracle_and_chain(torch_dev, case, precision):
    s = CASES[case]()
    assert 1 <= s.support_max <= 8
    modes = list(range(s.n)) if s.n <= 64 else sorted({0, s.n // 2 + 1, s.n - 1})
    print(f"[rows-first {precision}] {case}", flush=True)
    ref = {M: oracle.sym(s, M, modes=modes)["P"] for M in s.orders}
    bm = 32 if case.endswith("blocks32") else 0
    npf, Ps = B.compute(s, precision, block_modes=bm)                   # rows first
    npf_c, Pc = B.compute(s, precision, block_modes=bm, support_max=0)  # chain
    for M in s.orders:
        check(Ps[M][modes], ref[M], TOL[precision], f"P_{M}")
        check(Ps[M], Pc[M], 2 * TOL[precision], f"P_{M} vs chain")
    z = np.stack([s.delta * s.U[i, :] for i in modes])
    check(npf[:, modes].T, s.V[:, modes].T * (z + sum(ref.values())), TOL[precision], "NPF")


def test_too_small_support_bound_gives_nan(torch_dev):
    s = I.block_sparse_system(24, [2, 3], 8105)
    print("[rows-first bound too small]", flush=True)
    npf, Ps = B.compute(s, "fp64", support_max=3)        # rows involve 6 states
    assert np.isnan(npf).all()
    assert np.isnan(Ps[3]).all()                           # order 3 takes the route
