"""The error model behind the mixed-precision bound for plans beyond four orders (CPU only).

Emulates the arithmetic of the mixed paths in numpy: the chain of contractions in complex64
with every intermediate rounded, C read at the sorted representative of each index tuple
(so one rounding serves all of a tuple's orderings, as under symmetric packing), then the
divisor, quotient and reduction of Alg. 2 steps 5-19 in FP64.  The GPU test's bound is 2.5
times the largest emulated relative P error on this system (1.04e-6, order 5); the emulated
errors must stay within half of that bound, and the same
arithmetic without the shared rounding (each ordering rounded on its own) must be clearly
smaller -- which is what separates rounding replicated by the packing from a defect.
"""
import itertools
import math

import numpy as np

import oracle
from paper_2509_08968_amd import inputs as I
from tests.helpers import HIGH_ORDER_CASES, rel

BOUND = 2.6e-6          # the GPU test's bound for mixed paths beyond four orders
MARGIN = 2.0


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


def test_shared_rounding_explains_the_high_order_bound():
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
        assert e_shared <= BOUND / MARGIN, (M, e_shared)
        assert e_own < e_shared, (M, e_own, e_shared)
        assert e_own <= 5e-7, (M, e_own)
