"""Hash-generated derivative tensors and the kernel shapes above 64 states, on the GPU
through the C ABI.

- npf_hash_fill reproduces the generator's definition bit for bit;
- a hash-generated tensor gives bitwise the same NPFs as the same tensor stored;
- systems of 100 to 250 states, with output-mode blocks of 16 and 32 modes (several items
  per workgroup) and with the reduction's states split over workgroups (n > 128), match
  the oracle on sampled modes (P rows and NPF columns); so do systems of 300 and 351 states
  on the FP32 and FP64 paths;
- the n=200, orders 2-4 hash-generated workload at full size matches the stored oracle
  values of its sampled modes (P rows, NPF columns, and C and h on sampled tuples).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2509_08968_amd import binding as B
from paper_2509_08968_amd import inputs as I
from tests.helpers import check

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-6, "bf16x3": 1e-6}
GOLD200 = os.path.join(os.path.dirname(__file__), "golden", "hash200_modes.json")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    return torch, "cuda:0"


@pytest.mark.parametrize("n,M,k0,k1", [(37, 2, 0, 37), (200, 3, 5, 7), (9, 6, 0, 9), (200, 4, 199, 200)])
def test_hash_fill_bitwise(torch_dev, n, M, k0, k1):
    torch, dev = torch_dev
    print(f"[hash fill] n={n} M={M} rows {k0}:{k1}", flush=True)
    seed, scale = 977 + M, float(n) ** (-M / 2.0)
    U = math.comb(n + M - 1, M)
    out = torch.empty((k1 - k0) * U, dtype=torch.float64, device=dev)
    B.hash_fill(n, M, seed, scale, k0, k1, out)
    torch.cuda.synchronize()
    k = np.repeat(np.arange(k0, k1, dtype=np.uint64), U)
    r = np.tile(np.arange(U, dtype=np.uint64), k1 - k0)
    want = I.hash_value(seed, scale, M, k, r)
    assert np.array_equal(out.cpu().numpy().view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_hash_source_equals_stored_tensor(torch_dev, precision):
    s = I.hash_system(24, [2, 3, 4], 4501, materialize=True)
    print(f"[hash vs stored {precision}] n=24", flush=True)
    a, Pa = B.compute(s, precision, hash_source=True)
    b, Pb = B.compute(s, precision, hash_source=False)
    for M in s.orders:
        assert np.array_equal(Pa[M], Pb[M]), M
    assert np.array_equal(a, b)
    ref = {M: oracle.sym(s, M)["P"] for M in s.orders}
    for M in s.orders:
        check(Pa[M], ref[M], TOL[precision], f"P_{M}")


# name -> (builder, output modes per block or 0 for the planner's choice, precisions)
LARGE_CASES = {
    "n100-o3-dense-J16": (lambda: I.dense_system(100, [2, 3], 4601), 16, ["bf16x3", "fp64"]),
    "n100-o3-dense-J32": (lambda: I.dense_system(100, [2, 3], 4601), 32, ["bf16x3"]),
    "n150-o3-dense": (lambda: I.dense_system(150, [2, 3], 4602), 0, ["bf16x3", "fp32"]),
    "n200-o3-hash-J16": (lambda: I.hash_system(200, [2, 3], 4603), 16, ["bf16x3"]),
    "n250-o3-dense": (lambda: I.dense_system(250, [2, 3], 4604), 0, ["bf16x3"]),
    "n100-o4-hash-J48": (lambda: I.hash_system(100, [2, 3, 4], 4605), 48, ["bf16x3"]),
    # above 256 states: the FP32 and FP64 paths (tuple entries of 9 bits), NPCC-sized n = 351
    "n300-o3-hash": (lambda: I.hash_system(300, [2, 3], 4606), 0, ["fp64", "fp32"]),
    "n351-o3-hash": (lambda: I.hash_system(351, [2, 3], 4607), 0, ["fp64"]),
    "n300-o2-dense": (lambda: I.dense_system(300, [2], 4608), 0, ["fp64"]),
}
LARGE_PARAMS = [(c, p) for c, (_, _, ps) in sorted(LARGE_CASES.items()) for p in ps]


def _sampled(s, ref_modes, precision, block_modes, budget=0):
    ref = {M: oracle.sym(s, M, modes=ref_modes)["P"] for M in s.orders}
    npf, Ps = B.compute(s, precision, block_modes=block_modes, budget_bytes=budget)
    for M in s.orders:
        check(Ps[M][ref_modes], ref[M], TOL[precision], f"P_{M}")
    z = np.stack([s.delta * s.U[i, :] for i in ref_modes])
    npf_cols = s.V[:, ref_modes] * (z + sum(ref.values())).T
    check(npf[:, ref_modes].T, npf_cols.T, TOL[precision], "NPF")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("case,precision", LARGE_PARAMS)
def test_large_n_sampled_modes(torch_dev, case, precision):
    build, bm, _ = LARGE_CASES[case]
    s = build()
    modes = sorted({0, s.n // 2 + 1, s.n - 1})
    print(f"[large {precision}] {case} modes {modes}", flush=True)
    _sampled(s, modes, precision, bm)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["bf16x3", "fp32", "fp64"])
def test_workload_n200_o4_hash_sampled(torch_dev, precision):
    """n=200, orders 2-4, dense hash-generated tensors (never stored), in the configuration
    the benchmark times (its workspace budget); P rows and NPF columns of the sampled modes
    against the oracle values stored by tests/golden/make_hash200_golden.py."""
    import bench
    g = json.load(open(GOLD200))
    s = I.workload_hash200()
    modes = g["modes"]
    print(f"[n200-o4-hash {precision}] modes {modes}", flush=True)
    npf, Ps = B.compute(s, precision, conj=True,
                        budget_bytes=bench.budget_for("n200-o4-dense-hash", precision))
    cplx = lambda a: np.asarray(a)[..., 0] + 1j * np.asarray(a)[..., 1]
    for M in s.orders:
        check(Ps[M][modes], cplx(g["P"][str(M)]), TOL[precision], f"P_{M}")
    check(npf[:, modes].T, cplx(g["npf_columns"]), TOL[precision], "NPF")


CH_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hash200_ch.json")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["bf16x3", "fp32", "fp64"])
def test_workload_n200_o4_hash_c_and_h_sampled(torch_dev, precision):
    """C and h (Alg. 2 steps 1-11) of the n=200, orders 2-4 workload at full size, through a
    plan that selects four output modes and the staged entry points, on 1024 sampled sorted
    tuples per mode and order against stored oracle values (hash200_ch.json, written by
    make_hash200_ch_golden.py, which calls only the oracle)."""
    torch, dev = torch_dev
    g = json.load(open(CH_GOLDEN))
    s = I.workload_hash200()
    modes = g["modes"]
    d = B.upload_system(s, dev)
    plan = B.Plan(s.n, s.order_max, precision, s.eps, s.tau, s.delta, modes=modes)
    computed, _ = plan.modes()
    rows = [modes.index(m) for m in computed]        # golden row of each computed mode
    ws = plan.workspace(dev)
    cplx = lambda a: np.asarray(a)[..., 0] + 1j * np.asarray(a)[..., 1]
    print(f"[n200 C/h {precision}] modes {computed}", flush=True)
    for M in s.orders:
        e = g["orders"][str(M)]
        ranks = torch.tensor(e["ranks"], dtype=torch.int64, device=dev)
        C = torch.empty((len(computed), plan.unique_tuples[M]), dtype=torch.complex128, device=dev)
        plan.modal_contract(M, B.NPF_ALL_BLOCKS, d.tensors[M - 2], d.U, d.V, ws, C)
        torch.cuda.synchronize()
        Cs = C[:, ranks].cpu().numpy()
        plan.normal_form(M, B.NPF_ALL_BLOCKS, d.lam, C)
        torch.cuda.synchronize()
        hs = C[:, ranks].cpu().numpy()
        del C
        check(Cs, cplx(e["C"])[rows], TOL[precision], f"C_{M}")
        check(hs, cplx(e["h"])[rows], TOL[precision], f"h_{M}")
    plan.close()
