"""Argument checks of the C ABI entry points (host only).

Every case here is rejected by a host-side check before the entry point makes any HIP call,
so the calls carry placeholder device addresses.  The tests skip where a GPU is visible:
they exist for the validation logic, and a check that wrongly passed would otherwise
launch kernels on those placeholders.
"""
import ctypes

import pytest

from paper_2509_08968_amd import binding as B

FAKE = ctypes.c_void_p(0x10000)           # placeholder device address, never dereferenced


@pytest.fixture(scope="module")
def plan():
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-side argument checks are exercised where no GPU is visible")
    p = B.Plan(12, 3, "fp64")
    yield p
    p.close()


def _tensors(n_orders, over=None):
    ts = []
    for M in range(2, 2 + n_orders):
        d = dict(kind=B.SRC_DENSE, order=M, values=0x10000)
        d.update((over or {}).get(M, {}))
        t = B.NpfTensor()
        t.kind, t.order = d["kind"], d["order"]
        t.values = d["values"]
        for f in ("col_rank", "col_ptr", "row_k", "ncols", "nnz", "scale"):
            if f in d:
                setattr(t, f, d[f])
        ts.append(t)
    return (B.NpfTensor * n_orders)(*ts)


def _run(plan, tensors, U=FAKE, V=FAKE, lam=FAKE, ws=FAKE, ws_bytes=None):
    ws_bytes = plan.workspace_bytes if ws_bytes is None else ws_bytes
    return B.lib().npf_run(plan._h, tensors, U, V, lam, ws, ws_bytes, None, FAKE, FAKE)


def test_run_rejects_null_plan_and_arguments(plan):
    L = B.lib()
    t = _tensors(2)
    assert L.npf_run(None, t, FAKE, FAKE, FAKE, FAKE, 1, None, None, None) == B.NPF_E_INVALID
    assert _run(plan, None) == B.NPF_E_INVALID
    for kw in ("U", "V", "lam", "ws"):
        assert _run(plan, t, **{kw: None}) == B.NPF_E_INVALID, kw


def test_run_rejects_small_workspace(plan):
    assert _run(plan, _tensors(2), ws_bytes=plan.workspace_bytes - 1) == B.NPF_E_INVALID


@pytest.mark.parametrize("over,code", [
    ({3: dict(order=2)}, B.NPF_E_INVALID),                                  # order mismatch
    ({2: dict(values=0)}, B.NPF_E_INVALID),                                 # dense without values
    ({3: dict(kind=7)}, B.NPF_E_INVALID),                                   # unknown kind
    ({3: dict(kind=B.SRC_SPARSE, col_rank=0x10000, col_ptr=0x10000, row_k=0)}, B.NPF_E_INVALID),
    ({3: dict(kind=B.SRC_SPARSE, col_rank=0x10000, col_ptr=0x10000, row_k=0x10000,
              ncols=365, nnz=1)}, B.NPF_E_INVALID),                         # ncols > U_3(12) = 364
    ({2: dict(kind=B.SRC_SPARSE, col_rank=0x10000, col_ptr=0x10000, row_k=0x10000,
              ncols=-1)}, B.NPF_E_INVALID),
    ({3: dict(kind=B.SRC_HASH, values=0, scale=float("nan"))}, B.NPF_E_INVALID),
])
def test_run_rejects_bad_tensor_descriptors(plan, over, code):
    assert _run(plan, _tensors(2, over)) == code


def test_staged_entry_points_reject_bad_order_block_and_pointers(plan):
    L = B.lib()
    t = _tensors(2)
    ws = plan.workspace_bytes
    mc = lambda order, block, C=FAKE, ws_bytes=ws: L.npf_modal_contract(
        plan._h, order, block, ctypes.byref(t[max(0, min(order, 3) - 2)]), FAKE, FAKE, FAKE,
        ws_bytes, C, FAKE)
    assert mc(1, B.NPF_ALL_BLOCKS) == B.NPF_E_INVALID              # order below 2
    assert mc(4, B.NPF_ALL_BLOCKS) == B.NPF_E_INVALID              # order above order_max
    assert mc(2, 1) == B.NPF_E_INVALID                             # one block only (0)
    assert mc(2, -2) == B.NPF_E_INVALID
    assert mc(2, B.NPF_ALL_BLOCKS, C=None) == B.NPF_E_INVALID
    assert mc(2, B.NPF_ALL_BLOCKS, ws_bytes=ws - 1) == B.NPF_E_INVALID
    assert L.npf_normal_form(plan._h, 4, 0, FAKE, FAKE, FAKE) == B.NPF_E_INVALID
    assert L.npf_normal_form(plan._h, 2, 0, None, FAKE, FAKE) == B.NPF_E_INVALID
    assert L.npf_assemble(plan._h, 2, 5, FAKE, FAKE, FAKE, FAKE) == B.NPF_E_INVALID
    assert L.npf_assemble(plan._h, 2, 0, FAKE, None, FAKE, FAKE) == B.NPF_E_INVALID
    assert L.npf_finalize(plan._h, FAKE, FAKE, FAKE, None, FAKE) == B.NPF_E_INVALID
    assert L.npf_finalize(None, FAKE, FAKE, FAKE, FAKE, FAKE) == B.NPF_E_INVALID


@pytest.mark.parametrize("args", [
    (0, 2, 0, 1),          # n below 1
    (513, 2, 0, 1),        # n above 512
    (8, 1, 0, 8),          # order below 2
    (8, 7, 0, 8),          # order above 6
    (8, 2, 5, 3),          # k0 > k1
    (8, 2, 0, 9),          # k1 > n
])
def test_hash_fill_rejects_bad_ranges(plan, args):
    n, order, k0, k1 = args
    assert B.lib().npf_hash_fill(n, order, 1, 1.0, k0, k1, FAKE, FAKE) == B.NPF_E_INVALID


def test_hash_fill_rejects_null_output(plan):
    assert B.lib().npf_hash_fill(8, 2, 1, 1.0, 0, 8, None, FAKE) == B.NPF_E_INVALID
