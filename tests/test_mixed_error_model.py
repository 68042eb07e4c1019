"""The error model behind the mixed paths' order limit (CPU only).

Emulates the arithmetic of the mixed paths in numpy: the chain of contractions in complex64
with every intermediate rounded, C read at the sorted representative of each index tuple
(so one rounding serves all of a tuple's orderings, as under symmetric packing), then the
divisor, quotient and reduction of Alg. 2 steps 5-19 in FP64.  Through order 4 the emulated
relative P error stays well inside the mixed paths' 1e-6 bound; at order 5 the shared
rounding (up to 120 orderings per tuple) takes it to the bound itself, which is why plans
in FP32 or split-BF16 stop at order 4.  The same arithmetic with each ordering rounded on
its own is clearly smaller -- rounding replicated by the packing, not a defect.
"""
import itertools
import math

import numpy as np

import oracle
from paper_2509_08968_amd import inputs as I
from tests.helpers import HIGH_ORDER_CASES, rel

BOUND = 1e-6            # the mixed paths' bound on the relative error of P
MARGIN = 1.5


def _full(s, M):
    F = np.zeros((s.n,) + (s.n,) * M)
    for t in itertools.combinations_with_replacement(range(s.n), M):
        col = s.A[M][:, I.colex_rank(t)]
        for p in set(itertools.permutations(t)):
            F[(slice(None),) + p] = col
    return F


def _P_from_C(s, M, C):
    n = s.n
    D = -s.lam.reshape((n,) + (1,) * M)
    for i in range(M):
        sh = [1] * (M + 1)
        sh[i + 1] = n
        D = D + s.lam.reshape(sh)
    D = np.where(np.abs(D) < s.eps, s.eps, D)
    h = (C / D).reshape(n, -1)
    Z = np.ones((1, n), complex)
    for _ in range(M):
        Z = (Z[:, None, :] * (s.delta * s.U)[None, :, :]).reshape(-1, n)
    return -(h @ Z)


def test_shared_rounding_limits_mixed_paths_to_order_four():
    s = HIGH_ORDER_CASES["n18-o5-dense"]()
    n = s.n
    for M in s.orders:
        T = np.tensordot(s.U.astype(np.complex64), _full(s, M).astype(np.complex64), axes=(1, 0))
        for _ in range(M):
            T = np.tensordot(T, s.V.astype(np.complex64), axes=(1, 0)).astype(np.complex64)
        C = T.astype(np.complex128) / math.factorial(M)
        idx = np.indices((n,) * M).reshape(M, -1)
        rep = np.ravel_multi_index(tuple(np.sort(idx, axis=0)), (n,) * M)
        C_shared = C.reshape(n, -1)[:, rep].reshape(C.shape)
        ref = oracle.sym(s, M)["P"]
        e_shared = rel(_P_from_C(s, M, C_shared), ref)
        e_own = rel(_P_from_C(s, M, C), ref)
        if M <= 4:
            assert e_shared <= BOUND / MARGIN, (M, e_shared)
        else:
            assert e_shared > BOUND / MARGIN, (M, e_shared)
        assert e_own < e_shared, (M, e_own, e_shared)
        assert e_own <= 5e-7, (M, e_own)
