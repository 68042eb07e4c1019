"""Seeded synthetic inputs for the nonlinear-participation-factor (NPF) hot path.

This module only *makes data*: the spectrum and eigenvectors of a diagonalizable
system, its Jacobian, and real derivative tensors that are symmetric in their lower
indices, stored packed over sorted index tuples.  It holds none of the method's
arithmetic (no contraction, divisor, division or reduction), so both the HIP path and
the CPU oracle may take their inputs from here.

Packed storage (used everywhere in this project): for an order-M tensor AN^k_{a1..aM}
that is symmetric in (a1..aM), entry (k, sorted tuple t_1 <= ... <= t_M) lives at
``A[k, rank(t)]`` where ``rank(t) = sum_{i=1..M} binom(t_i + i - 1, i)`` (colex rank,
0-based states, 1-based positions).  The rank is a bijection onto
``[0, binom(n + M - 1, M))`` and is prefix-stable in n.  The stored value is the
derivative value (the Taylor coefficient times M!), matching eq. (1) read as a
derivative expansion and Alg. 2 step 4, which divides by N!.

Hash-generated tensors: for systems too large to store, A_M is defined by a counter-based
generator instead of stored values (see ``hash_value``); the GPU library generates the
entries it needs on the device and the CPU oracle generates them on the host, each from
the generator's published definition.  The numpy version here materialises small cases.

The workloads follow the paper's setting (Section III: power-system models of 6 to
4251 states, orders 2 to 4).  The paper's systems are not available, so seeded
stand-ins of the same shapes are generated; the recipe of each is stated in the
builder's docstring.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

BASE_SEED = 20250908


# ----------------------------------------------------------------------------- packing
def n_sorted(n: int, m: int) -> int:
    """Number of sorted m-tuples over n states, binom(n + m - 1, m)."""
    if m == 0:
        return 1
    return math.comb(n + m - 1, m)


def colex_rank(t) -> int:
    """Colex rank of a sorted tuple (0-based values, 1-based positions)."""
    return sum(math.comb(int(x) + i, i + 1) for i, x in enumerate(t))


def sorted_tuples(n: int, m: int) -> np.ndarray:
    """All sorted m-tuples over range(n) as an int array [binom(n+m-1,m), m], in colex order."""
    if m == 0:
        return np.zeros((1, 0), dtype=np.int64)
    tups = list(itertools.combinations_with_replacement(range(n), m))
    tups.sort(key=lambda t: t[::-1])
    return np.asarray(tups, dtype=np.int64).reshape(-1, m)


# ----------------------------------------------------------------------------- system
@dataclasses.dataclass
class System:
    """One operating point: spectrum, eigenvectors and packed derivative tensors.

    lam   complex128 [n]        eigenvalues (mode order = output order)
    V     complex128 [n, n]     right eigenvectors as columns, Phi[state, mode]
    U     complex128 [n, n]     left eigenvectors as rows, Psi[mode, state], U @ V = I
    A1    float64    [n, n]     Jacobian, Re(V diag(lam) U)
    A     {M: float64 [n, binom(n+M-1, M)]}  packed derivative tensors, M >= 2
    support {M: int64 [s]}      sorted union of ranks that may be nonzero (None = dense)
    hashed  {M: (seed, scale)}  orders whose A_M is hash-generated (A[M] is None)
    support_max                 most distinct states in one row k of a sparse A_M (0: dense)
    """

    name: str
    n: int
    lam: np.ndarray
    V: np.ndarray
    U: np.ndarray
    A1: np.ndarray
    A: Dict[int, np.ndarray]
    support: Dict[int, Optional[np.ndarray]]
    eps: float = 1e-9
    tau: float = 1e-2
    delta: float = 1.0
    hashed: Dict[int, Tuple[int, float]] = dataclasses.field(default_factory=dict)
    support_max: int = 0        # most distinct states one row k of a sparse A_M involves

    @property
    def orders(self) -> List[int]:
        return sorted(self.A)

    @property
    def order_max(self) -> int:
        return max(self.A) if self.A else 1


MAX_DRAWS = 1000    # redraws of a spectrum before a generator gives up


def _spectrum(n: int, rng: np.random.Generator, min_gap: float = 1e-3) -> np.ndarray:
    """Conjugate pairs: Re ~ U[-2, -0.05], Im ~ U[0.5, 10]; an odd n gets one real root."""
    for _ in range(MAX_DRAWS):
        lam = np.empty(n, dtype=np.complex128)
        for m in range(n // 2):
            re = rng.uniform(-2.0, -0.05)
            im = rng.uniform(0.5, 10.0)
            lam[2 * m] = complex(re, im)
            lam[2 * m + 1] = complex(re, -im)
        if n % 2:
            lam[n - 1] = complex(rng.uniform(-2.0, -0.05), 0.0)
        if _min_gap(lam) >= min_gap:
            return lam
    raise ValueError(f"no spectrum of {n} eigenvalues at least {min_gap} apart in {MAX_DRAWS} draws")


def _min_gap(lam: np.ndarray) -> float:
    d = np.abs(lam[:, None] - lam[None, :])
    np.fill_diagonal(d, np.inf)
    return float(d.min()) if lam.size > 1 else np.inf


def _eigvecs(n: int, rng: np.random.Generator) -> np.ndarray:
    """Columns (v, conj v) per pair with Re, Im ~ N(0, 1); a real column for an odd n."""
    V = np.empty((n, n), dtype=np.complex128)
    for m in range(n // 2):
        v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        V[:, 2 * m] = v
        V[:, 2 * m + 1] = np.conj(v)
    if n % 2:
        V[:, n - 1] = rng.standard_normal(n)
    return V


def _finish(name, n, lam, V, A, support, **kw) -> System:
    U = np.linalg.inv(V)
    A1 = np.real(V @ np.diag(lam) @ U).copy()
    return System(name=name, n=n, lam=lam, V=V, U=U, A1=A1, A=A, support=support, **kw)


def dense_tensor(n: int, M: int, scale: float, rng: np.random.Generator) -> np.ndarray:
    """Packed dense symmetric tensor with i.i.d. N(0, 1) * scale entries per sorted tuple."""
    return rng.standard_normal((n, n_sorted(n, M))) * scale


def block_sets(n: int, block: int = 4, extra: int = 2) -> List[List[int]]:
    """Per-state support S(k): k's block of ``block`` states plus the first ``extra``
    states of the next block (cyclic).  The last block is shorter when block does not
    divide n."""
    starts = list(range(0, n, block))
    blocks = [list(range(s, min(s + block, n))) for s in starts]
    sets = []
    for b, blk in enumerate(blocks):
        nxt = blocks[(b + 1) % len(blocks)]
        s = sorted(set(blk) | set(nxt[:extra]))
        sets.extend([s] * len(blk))
    return sets


def block_sparse_tensor(n: int, M: int, rng: np.random.Generator, block: int = 4,
                        extra: int = 2, scale: float = 1.0):
    """Machine-like block-sparse derivative tensor: row k depends only on S(k).

    Nonzeros are N(0, 1) * scale on the sorted M-tuples of S(k), drawn k by k in colex
    order of the tuples.  Returns (packed dense array with zeros, sorted union support).
    """
    A = np.zeros((n, n_sorted(n, M)))
    sets = block_sets(n, block, extra)
    support = set()
    for k in range(n):
        tups = sorted(itertools.combinations_with_replacement(sets[k], M), key=lambda t: t[::-1])
        ranks = [colex_rank(t) for t in tups]
        A[k, ranks] = rng.standard_normal(len(ranks)) * scale
        support.update(ranks)
    return A, np.asarray(sorted(support), dtype=np.int64)


def dense_system(n: int, orders, seed: int, name: str = "dense", scale_pow: float = 0.5,
                 **kw) -> System:
    """Dense symmetric A_M with entries N(0,1) / n^(M * scale_pow)."""
    rng = np.random.default_rng(seed)
    lam = _spectrum(n, rng)
    V = _eigvecs(n, rng)
    A = {M: dense_tensor(n, M, float(n) ** (-M * scale_pow), rng) for M in orders if M >= 2}
    return _finish(name, n, lam, V, A, {M: None for M in A}, **kw)


def block_sparse_system(n: int, orders, seed: int, name: str = "block-sparse", **kw) -> System:
    """Block-sparse A_M (4-state blocks plus 2 coupling states), entries N(0, 1)."""
    rng = np.random.default_rng(seed)
    lam = _spectrum(n, rng)
    V = _eigvecs(n, rng)
    A, S = {}, {}
    for M in orders:
        if M >= 2:
            A[M], S[M] = block_sparse_tensor(n, M, rng)
    smax = max(len(x) for x in block_sets(n))
    return _finish(name, n, lam, V, A, S, support_max=smax, **kw)


def resonant_system(n: int, orders, seed: int, n_res2: int = 4, n_res3: int = 4,
                    eta_lo: float = 1e-6, eta_hi: float = 1e-4, name: str = "dense-resonant",
                    **kw) -> System:
    """Dense system with planted near resonances (small divisors).

    ``n_res2`` target pairs get lambda_j = lambda_p + lambda_q + eta and ``n_res3`` get
    lambda_j = lambda_p + lambda_q + lambda_r + eta, with distinct upper-half-plane
    sources that are not targets, |eta| log-uniform in [eta_lo, eta_hi] and a uniform
    phase; the conjugate partner follows.  A_M entries are N(0,1) / n^(M/2).
    """
    n_t = n_res2 + n_res3
    if n_t + 2 * n_res2 + 3 * n_res3 > n // 2:
        raise ValueError("not enough conjugate pairs for distinct targets and sources")
    rng = np.random.default_rng(seed)
    for _ in range(MAX_DRAWS):
        lam = _spectrum(n, rng)
        pairs = rng.permutation(n // 2)
        targets, sources = pairs[:n_t], list(pairs[n_t:])
        cursor = 0
        for idx, m in enumerate(targets):
            width = 2 if idx < n_res2 else 3
            src = sources[cursor:cursor + width]
            cursor += width
            eta = np.exp(rng.uniform(np.log(eta_lo), np.log(eta_hi))) * np.exp(
                1j * rng.uniform(0.0, 2.0 * np.pi))
            val = sum(lam[2 * s] for s in src) + eta
            lam[2 * m] = val
            lam[2 * m + 1] = np.conj(val)
        if _min_gap(lam) >= 1e-3 and np.all(np.abs(lam.imag) > 0):
            break
    else:
        raise ValueError(f"no resonant spectrum with distinct eigenvalues in {MAX_DRAWS} draws")
    V = _eigvecs(n, rng)
    A = {M: dense_tensor(n, M, float(n) ** (-M / 2.0), rng) for M in orders if M >= 2}
    return _finish(name, n, lam, V, A, {M: None for M in A}, **kw)


CLAMP_EPS = 2.0 ** -17          # the clamp threshold of the clamp systems (about 7.6e-6)


def clamp_system(n: int, orders, seed: int, eps: float = CLAMP_EPS, name: str = "clamp",
                 **kw) -> System:
    """Dense system whose small divisors sit exactly at, just below and just above the clamp
    threshold ``eps`` of Alg. 2 step 9, with every divisor exact in FP64.

    Eigenvalues are conjugate pairs on the dyadic grid 2^-6 (Re in [-2, -0.0625], Im in
    [0.5, 10]).  Four target pairs are then set, from distinct non-target sources, to
        lam_j = lam_p + lam_q                 (order-2 divisor exactly 0: clamped),
        lam_j = lam_p + lam_q + lam_r         (order-3 divisor exactly 0: clamped),
        lam_j = lam_p + lam_q - (15/16) eps   (|D| just below eps: clamped),
        lam_j = lam_p + lam_q - (17/16) eps   (|D| just above eps: not clamped),
    and, when order 4 is present, a fifth to lam_p + lam_q + lam_r + lam_s (order-4 divisor
    exactly 0); the conjugate partner follows.  These values need at most 27 significant bits, so
    the sums of up to four eigenvalues and the divisors are exact in FP64 whatever the
    summation order.  A_M entries are N(0, 1) / n^(M/2), eps is the system's clamp."""
    o4 = 4 in orders
    if n // 2 < (18 if o4 else 13):
        raise ValueError("clamp systems need 13 conjugate pairs (18 with order 4)")
    rng = np.random.default_rng(seed)
    grid = 2.0 ** -6
    for _ in range(MAX_DRAWS):
        lam = np.empty(n, dtype=np.complex128)
        for m in range(n // 2):
            v = complex(-grid * rng.integers(4, 129), grid * rng.integers(32, 641))
            lam[2 * m], lam[2 * m + 1] = v, np.conj(v)
        if n % 2:
            lam[n - 1] = complex(-grid * rng.integers(4, 129), 0.0)
        pairs = rng.permutation(n // 2)
        nt = 5 if o4 else 4
        targets, src = pairs[:nt], [int(x) for x in pairs[nt:nt + 13]]
        plans = [(src[0:2], 0.0), (src[2:5], 0.0), (src[5:7], -eps * 15 / 16),
                 (src[7:9], -eps * 17 / 16)] + ([(src[9:13], 0.0)] if o4 else [])
        for m, (ss, off) in zip(targets, plans):
            v = lam[2 * ss[0]]
            for x in ss[1:]:
                v = v + lam[2 * x]
            v = v + off
            lam[2 * m], lam[2 * m + 1] = v, np.conj(v)
        if _min_gap(lam) >= 1e-3:
            break
    else:
        raise ValueError(f"no clamp spectrum with distinct eigenvalues in {MAX_DRAWS} draws")
    V = _eigvecs(n, rng)
    A = {M: dense_tensor(n, M, float(n) ** (-M / 2.0), rng) for M in orders if M >= 2}
    return _finish(name, n, lam, V, A, {M: None for M in A}, eps=eps, **kw)


def poly_field(n: int, orders, seed: int, terms_per_eq: int = 6, max_degree: int = None,
               x_eq=None, scale: float = 0.5, spectrum_seed: int = None):
    """A sparse polynomial vector field x' = f(x) with f(0) = 0: the linear part is the
    Jacobian A1 = Re(V diag(lam) V^-1) of a seeded spectrum (as for the other systems), and
    every equation k gets ``terms_per_eq`` monomials of each degree in ``orders`` over
    seeded variables (with repetition), coefficients N(0, 1) * scale^degree.  Returns the
    terms as arrays (eq [T], coef [T], var [T, D] padded with -1, D = max degree) sorted by
    equation, the CSR offsets eq_ptr [n+1], the expansion point x_eq (None = 0) and the
    spectrum (lam, V, U = V^-1)."""
    rng = np.random.default_rng(seed)
    lam = _spectrum(n, rng)
    V = _eigvecs(n, rng)
    U = np.linalg.inv(V)
    A1 = np.real(V @ np.diag(lam) @ U)
    D = max(max(orders), 1) if max_degree is None else max_degree
    eq, coef, var = [], [], []
    for k in range(n):
        for a in range(n):
            eq.append(k); coef.append(A1[k, a]); var.append([a] + [-1] * (D - 1))
        for d in sorted(orders):
            for _ in range(terms_per_eq):
                vs = sorted(int(x) for x in rng.integers(0, n, d))
                eq.append(k); coef.append(rng.standard_normal() * scale ** d)
                var.append(vs + [-1] * (D - d))
    eq = np.asarray(eq, np.int32)
    eq_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(eq, minlength=n), out=eq_ptr[1:])
    return {"n": n, "eq": eq, "coef": np.asarray(coef), "var": np.asarray(var, np.int32),
            "eq_ptr": eq_ptr, "x_eq": None if x_eq is None else np.asarray(x_eq, np.float64),
            "lam": lam, "V": V, "U": U, "A1": A1}


# ----------------------------------------------------------------------------- hash tensors
SPLITMIX_GAMMA = 0x9E3779B97F4A7C15
HASH_SQRT3 = 1.7320508075688772


def hash_counter(M: int, k, r):
    """Counter of entry (order M, state k, colex rank r): (M << 49) | (k << 40) | r.
    Valid for M < 8, k < 512 and r < 2^40."""
    return (np.uint64(M) << np.uint64(49)) | (np.asarray(k, dtype=np.uint64) << np.uint64(40)) \
        | np.asarray(r, dtype=np.uint64)


def splitmix64(seed: int, idx) -> np.ndarray:
    """Output number ``idx`` (0-based) of SplitMix64 started at ``seed`` (Steele, Lea and
    Flood, OOPSLA 2014): z = seed + (idx + 1) * gamma, then the variant-13 finaliser
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
    z ^= z >> 31 (all mod 2^64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(idx, dtype=np.uint64) + np.uint64(1)) * np.uint64(SPLITMIX_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def hash_value(seed: int, scale: float, M: int, k, r) -> np.ndarray:
    """Entry A_M[k, r] of a hash-generated tensor.

    w = splitmix64(seed, counter(M, k, r)); its four 16-bit fields f_q give four uniforms
    (f_q + 1/2) / 2^16 whose sum minus 2 has mean 0 and variance 1/3 (Irwin-Hall), so
    x = (S - 131070) * 2^-16 with S = f_0 + f_1 + f_2 + f_3 (exact), and
    A = (x * sqrt(3)) * scale with two IEEE roundings in that order.  No transcendental
    function is involved, so every implementation reproduces the bits."""
    w = splitmix64(seed, hash_counter(M, k, r))
    S = np.zeros(w.shape, dtype=np.int64)
    for q in range(4):
        S += ((w >> np.uint64(16 * q)) & np.uint64(0xFFFF)).astype(np.int64)
    x = (S - 131070).astype(np.float64) * 2.0 ** -16
    return (x * HASH_SQRT3) * np.float64(scale)


def hash_tensor(n: int, M: int, seed: int, scale: float) -> np.ndarray:
    """Packed [n, binom(n+M-1, M)] materialisation of a hash-generated tensor (small n)."""
    U = n_sorted(n, M)
    k = np.repeat(np.arange(n, dtype=np.uint64), U)
    r = np.tile(np.arange(U, dtype=np.uint64), n)
    return hash_value(seed, scale, M, k, r).reshape(n, U)


def hash_system(n: int, orders, seed: int, name: str = "hash", materialize: bool = False,
                **kw) -> System:
    """Dense system whose A_M are hash-generated with scale n^(-M/2) and generator seed
    ``seed + M``; spectrum and eigenvectors as for the other systems.  With
    ``materialize`` the packed tensors are also built (small n only)."""
    rng = np.random.default_rng(seed)
    lam = _spectrum(n, rng)
    V = _eigvecs(n, rng)
    hashed = {M: (int(seed + M), float(n) ** (-M / 2.0)) for M in orders if M >= 2}
    A = {M: (hash_tensor(n, M, *hashed[M]) if materialize else None) for M in hashed}
    return _finish(name, n, lam, V, A, {M: None for M in A}, hashed=hashed, **kw)


# ----------------------------------------------------------------------------- workloads
def workload_small() -> System:
    """n=10, orders 1-2: five conjugate pairs, dense A2 ~ N(0,1)/n."""
    return dense_system(10, [2], BASE_SEED + 0, name="n10-o2-dense", scale_pow=0.5)


def workload_sparse64() -> System:
    """n=64, orders 2-3, block-sparse A2/A3 (each row depends on <= 6 states)."""
    return block_sparse_system(64, [2, 3], BASE_SEED + 1, name="n64-o3-blocksparse")


def workload_dense128() -> System:
    """n=128, orders 2-4, dense A_M ~ N(0,1)/n^(M/2), 8 planted near resonances."""
    return resonant_system(128, [2, 3, 4], BASE_SEED + 2, name="n128-o4-dense-resonant")


def workload_hash200() -> System:
    """n=200, orders 2-4, dense A_M ~ Irwin-Hall(4) / n^(M/2), hash-generated (A_4 alone
    would be 110 GB in FP64)."""
    return hash_system(200, [2, 3, 4], BASE_SEED + 4, name="n200-o4-dense-hash")


def workload_batch(count: int = 256, seed: int = BASE_SEED + 3) -> List[System]:
    """``count`` block-sparse systems, n uniform over even values in [32, 160], orders 2-3."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.arange(32, 161, 2), size=count)
    return [block_sparse_system(int(n), [2, 3], seed * 1000 + i, name=f"batch{i}-n{n}")
            for i, n in enumerate(ns)]


WORKLOADS = {
    "n10-o2-dense": workload_small,
    "n64-o3-blocksparse": workload_sparse64,
    "n128-o4-dense-resonant": workload_dense128,
    "n200-o4-dense-hash": workload_hash200,
}


# ----------------------------------------------------------------------------- sparse views
def sparse_entries(A: np.ndarray, support: Optional[np.ndarray] = None):
    """(k, rank, value) triples of the nonzeros of a packed tensor, ordered by rank then k."""
    if support is None:
        k, r = np.nonzero(A)
    else:
        sub = A[:, support]
        k, ri = np.nonzero(sub)
        r = support[ri]
    order = np.lexsort((k, r))
    k, r = k[order], r[order]
    return k.astype(np.int64), r.astype(np.int64), A[k, r].astype(np.float64)
