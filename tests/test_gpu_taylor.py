"""Derivative tensors on the device (the numerical Taylor expansion of Alg. 1), through the
C ABI: npf_taylor_fill against the oracle's binomial expansion of the same polynomial field,
element by element, at x* = 0 and x* != 0, orders 1-6, one batch and several; then the whole
hot path on the device-filled tensors against the oracle's NPFs on its own tensors."""
import ctypes
import math

import numpy as np
import pytest

import oracle
from paper_2509_08968_amd import binding as B
from paper_2509_08968_amd import inputs as I
from tests.helpers import check

pytestmark = pytest.mark.gpu

# Error bound of the fill relative to max(1, largest entry of the tensor).  At x* = 0 an
# entry is a coefficient times an integer sum; at x* != 0 the alternating sums and the
# Lagrange extraction at nodes up to |s| = 3 cancel values up to (|x*| + 3 M)^d, so the
# error grows with the degree: a replay of the same arithmetic in FP64 on the CPU stays
# below 3e-15 for the fields here (degree <= 6), and 1e-12 keeps a wide margin.
FILL_TOL = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.lib()
    return torch, "cuda:0"


def _fill(torch, dev, field, M, k0=0, k1=None, batch_rows=0, init=float("nan")):
    poly = B.DevicePoly(field, dev)
    n = field["n"]
    k1 = n if k1 is None else k1
    UM = math.comb(n + M - 1, M)
    out = torch.full(((k1 - k0) * UM,), init, dtype=torch.float64, device=dev)
    step = batch_rows or (k1 - k0) or 1
    for a in range(k0, k1, step):
        b = min(k1, a + step)
        B.taylor_fill(poly, M, a, b, out[(a - k0) * UM:(b - k0) * UM])
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(k1 - k0, UM)


def _expect_close(got, ref, what):
    scale = max(1.0, float(np.abs(ref).max()))
    err = float(np.abs(got - ref).max())
    print(f"  {what}: max|diff| {err:.3e}, max|A| {np.abs(ref).max():.3e}", flush=True)
    assert np.all(np.isfinite(got)), what
    assert err <= FILL_TOL * scale, (what, err, scale)


FIELDS = {
    "n7-d5-origin": dict(n=7, orders=[2, 3, 4, 5], seed=1401, terms_per_eq=5),
    "n7-d5-shifted": dict(n=7, orders=[2, 3, 4, 5], seed=1402, terms_per_eq=5, shifted=True),
    "n6-d6-shifted": dict(n=6, orders=[2, 4, 6], seed=1403, terms_per_eq=3, shifted=True),
    "n40-d4-shifted": dict(n=40, orders=[2, 3, 4], seed=1404, terms_per_eq=6, shifted=True),
}


def _field(spec):
    spec = dict(spec)
    shifted = spec.pop("shifted", False)
    x_eq = None
    if shifted:
        x_eq = np.random.default_rng(spec["seed"] + 7).standard_normal(spec["n"]) * 0.5
    return I.poly_field(x_eq=x_eq, **spec)


@pytest.mark.parametrize("name", sorted(FIELDS))
def test_taylor_fill_matches_oracle(torch_dev, name):
    torch, dev = torch_dev
    field = _field(FIELDS[name])
    n = field["n"]
    top = max(FIELDS[name]["orders"])
    print(f"[taylor fill] {name}", flush=True)
    for M in range(1, min(top, B.NPF_MAX_ORDER) + 1):
        if n > 10 and M > 4:
            continue
        ref = oracle.poly_tensor(field, n, M)
        got = _fill(torch, dev, field, M)
        _expect_close(got, ref, f"A_{M}")


def test_taylor_fill_jacobian_at_origin(torch_dev):
    """Order 1 at x* = 0 is the linear part of the field, the Jacobian A1."""
    torch, dev = torch_dev
    field = I.poly_field(30, [2, 3], 1405)
    got = _fill(torch, dev, field, 1)
    assert np.allclose(got, field["A1"], rtol=0, atol=1e-15 * np.abs(field["A1"]).max())


def test_taylor_fill_batches_equal_one_call(torch_dev):
    """Row batches (the index ranges of Alg. 1) give bitwise the rows of one call."""
    torch, dev = torch_dev
    field = _field(FIELDS["n40-d4-shifted"])
    for M in (2, 3):
        whole = _fill(torch, dev, field, M)
        parts = _fill(torch, dev, field, M, batch_rows=7)
        assert np.array_equal(whole, parts)
        mid = _fill(torch, dev, field, M, k0=11, k1=29)
        assert np.array_equal(mid, whole[11:29])


def test_taylor_fill_edges(torch_dev):
    torch, dev = torch_dev
    # a field without terms of the order's degree (and one equation without any term)
    field = I.poly_field(5, [2], 1406, terms_per_eq=2)
    field["eq_ptr"] = field["eq_ptr"].copy()
    field["eq_ptr"][1] = 0                  # equation 0 without terms
    A3 = _fill(torch, dev, field, 3)
    assert np.array_equal(A3, np.zeros_like(A3))
    # n = 1: f = 2 x + 3 x^2 - x^3 about x* = 0.5: f'' = 6 - 6 x* = 3, f''' = -6
    one = {"n": 1, "eq": np.zeros(3, np.int32), "coef": np.array([2.0, 3.0, -1.0]),
           "var": np.array([[0, -1, -1], [0, 0, -1], [0, 0, 0]], np.int32),
           "eq_ptr": np.array([0, 3], np.int64), "x_eq": np.array([0.5])}
    assert _fill(torch, dev, one, 2)[0, 0] == 3.0
    assert _fill(torch, dev, one, 3)[0, 0] == -6.0
    assert _fill(torch, dev, one, 4)[0, 0] == 0.0
    # a variable outside [0, n) turns its row into NaN; the other rows are untouched
    bad = I.poly_field(4, [2], 1407, terms_per_eq=2)
    bad["var"] = bad["var"].copy()
    q = int(bad["eq_ptr"][2])            # first term of equation 2
    bad["var"][q, 0] = 4
    got = _fill(torch, dev, bad, 2, init=0.0)
    assert np.all(np.isnan(got[2]))
    ok = np.ones(4, bool)
    ok[2] = False
    assert np.all(np.isfinite(got[ok]))
    # argument errors are refused before anything runs
    poly = B.DevicePoly(field, dev)
    out = torch.zeros(64, dtype=torch.float64, device=dev)
    for args in [(0, 2, 0, 1), (5, 7, 0, 1), (5, 2, 3, 2), (5, 2, 0, 6)]:
        n, M, k0, k1 = args
        rc = B.lib().npf_taylor_fill(n, M, ctypes.byref(poly.desc), k0, k1, out.data_ptr(), None)
        assert rc == B.NPF_E_INVALID, args
    assert B.lib().npf_taylor_fill(5, 2, None, 0, 1, out.data_ptr(), None) == B.NPF_E_INVALID


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("shifted", [False, True])
def test_npfs_from_device_tensors(torch_dev, precision, shifted):
    """Model -> tensors -> NPFs: the hot path on the tensors npf_taylor_fill wrote (in row
    batches) against the oracle's NPFs on the tensors of its own expansion, same spectrum."""
    torch, dev = torch_dev
    n, orders = 24, [2, 3, 4]
    x_eq = np.random.default_rng(1408).standard_normal(n) * 0.3 if shifted else None
    field = I.poly_field(n, orders, 1409, terms_per_eq=6, x_eq=x_eq)
    sysm = I.System(name="poly", n=n, lam=field["lam"], V=field["V"], U=field["U"],
                    A1=field["A1"], A={M: oracle.poly_tensor(field, n, M) for M in orders},
                    support={M: None for M in orders}, delta=0.2)
    print(f"[taylor npf] {precision} shifted={shifted}", flush=True)
    npf_ref, Ps_ref = oracle.npf(sysm)
    poly = B.DevicePoly(field, dev)
    tens = [B.taylor_tensor(poly, M, dev, batch_rows=5) for M in orders]
    c128 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.complex128)).to(dev)
    plan = B.Plan(n, max(orders), precision, sysm.eps, sysm.tau, sysm.delta)
    ws = plan.workspace(dev)
    P = torch.zeros((len(orders), n, n), dtype=torch.complex128, device=dev)
    npf = torch.zeros((n, n), dtype=torch.complex128, device=dev)
    plan.run(tens, c128(sysm.U), c128(sysm.V), c128(sysm.lam), ws, P, npf)
    torch.cuda.synchronize()
    tol = 1e-10 if precision == "fp64" else 1e-6
    for i, M in enumerate(orders):
        check(P[i].cpu().numpy(), Ps_ref[M], tol, f"P_{M}")
    check(npf.cpu().numpy().T, npf_ref.T, tol, "NPF")
    plan.close()
