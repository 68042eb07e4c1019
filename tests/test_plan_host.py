"""Host-side checks of the library (no GPU): exported symbols, Alg. 1 against the paper's
Tables II/III, and the planner's validation and block sizing."""
import ctypes
import json
import os
import re

import numpy as np
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
    (dict(n=513, order_max=2), B.NPF_E_UNSUPPORTED),
    (dict(n=257, order_max=2, precision="bf16x3"), B.NPF_E_UNSUPPORTED),
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
    # FP32 and FP64 plans go to 512 states (tuple entries of 9 bits)
    for prec in ("fp32", "fp64"):
        p = B.Plan(512, 3, prec, budget_bytes=64 << 30)
        assert p.unique_tuples[3] == 514 * 513 * 512 // 6
        assert p.block_modes * p.n_blocks >= 512
        p.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mixed_plans_refuse_orders_above_four(precision):
    """The FP32 and split-BF16 paths meet their 1e-6 bound up to order 4 only: plans of
    five or six orders in those precisions are refused, FP64 plans accepted."""
    for N in (5, 6):
        with pytest.raises(B.NpfError) as e:
            B.Plan(12, N, precision)
        assert e.value.code == B.NPF_E_UNSUPPORTED
        B.Plan(12, N, "fp64").close()
    B.Plan(12, 4, precision).close()


def test_output_modes_and_conjugate_pairs():
    """Output modes {1, 4, 5} of six modes paired (0,1), (2,3), (4,5): mode 1 is computed
    (its partner is not requested), 4 is computed and fills 5."""
    conj = [1, 0, 3, 2, 5, 4]
    p = B.Plan(6, 3, "fp64", modes=[4, 1, 5], conj_of=conj)
    assert p.output_modes == 3 and p.computed_modes == 2
    assert p.modes() == ([1, 4], [-1, 5])
    p.close()
    lam = np.empty(64, complex)
    lam[0::2], lam[1::2] = np.arange(32) + 2j, np.arange(32) - 2j
    q = B.Plan(64, 3, "bf16x3", conj_of=B.conj_pairs(lam))
    assert q.computed_modes == 32 and q.output_modes == 64
    assert q.modes()[1] == list(range(1, 64, 2))
    full = B.Plan(64, 3, "bf16x3")
    assert full.computed_modes == 64 and full.modes()[1] == [-1] * 64
    assert q.workspace_bytes < full.workspace_bytes


@pytest.mark.parametrize("kw,msg", [
    (dict(modes=[1, 1]), "twice"), (dict(modes=[6]), "outside"), (dict(modes=[-1]), "outside"),
    (dict(conj_of=[1, 0, 3, 2, 5, 5]), "involution"), (dict(conj_of=[1, 2, 0, 3, 4, 5]), "involution"),
])
def test_output_mode_lists_are_validated(kw, msg):
    with pytest.raises(B.NpfError) as e:
        B.Plan(6, 2, "fp64", **kw)
    assert e.value.code == B.NPF_E_INVALID and msg in str(e.value)


def test_host_copies_check_preconditions():
    """Psi Phi = I and the conjugate pairing are checked when host copies are given."""
    from paper_2509_08968_amd import inputs as I
    s = I.dense_system(10, [2], 55)
    conj = B.conj_pairs(s.lam)
    B.Plan(10, 2, "fp64", conj_of=conj, check=(s.U, s.V, s.lam)).close()
    with pytest.raises(B.NpfError, match="identity"):
        B.Plan(10, 2, "fp64", check=(s.U.T.copy(), s.V, None))
    bad = s.lam.copy()
    bad[1] += 1e-3
    with pytest.raises(B.NpfError, match="eigenvalues"):
        B.Plan(10, 2, "fp64", conj_of=conj, check=(None, None, bad))
    V2 = s.V.copy()
    V2[:, 1] *= 1j                           # still an eigenvector, no longer the conjugate
    U2 = np.linalg.inv(V2)
    with pytest.raises(B.NpfError, match="right eigenvectors"):
        B.Plan(10, 2, "fp64", conj_of=conj, check=(U2, V2, s.lam))
    with pytest.raises(B.NpfError, match="convention"):
        prob = B.NpfProblem(10, 2, 0, 1e-9, 1e-2, 1.0, 0, 0, 0, 0, 7)
        h = ctypes.c_void_p()
        B._check(B.lib().npf_plan_create(ctypes.byref(prob), ctypes.byref(h)), "npf_plan_create")


def test_conj_pairs_of_a_spectrum():
    lam = np.array([1 + 2j, 3 + 0j, 1 - 2j, -1 - 1j, -1 + 1j])
    assert B.conj_pairs(lam).tolist() == [2, 1, 0, 4, 3]
    with pytest.raises(ValueError):
        B.conj_pairs(np.array([1 + 2j, 1 + 1j]))
