"""ctypes binding of libnpf.so (the C ABI in include/npf.h).

Argument marshalling only: torch supplies device memory and the HIP stream, every step of
the hot path runs in the library's HIP kernels.  Importing this module does not need a
GPU; loading the library fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnpf.so")

NPF_OK, NPF_E_INVALID, NPF_E_BUDGET, NPF_E_DEVICE, NPF_E_UNSUPPORTED = 0, 1, 2, 3, 4
NPF_MAX_ORDER = 6
NPF_ALL_BLOCKS = -1
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
SRC_DENSE, SRC_SPARSE, SRC_HASH = 0, 1, 2

EXPORTED = [
    "npf_plan_create", "npf_plan_info", "npf_plan_destroy", "npf_modal_contract",
    "npf_normal_form", "npf_assemble", "npf_finalize", "npf_run", "npf_alg1_batches",
    "npf_plan_profile", "npf_plan_kernel_times", "npf_error_string", "npf_last_error",
    "npf_hash_fill", "npf_batch_create", "npf_batch_info", "npf_batch_destroy",
    "npf_batch_run", "npf_batch_tune", "npf_batch_launches", "npf_batch_time",
    "npf_plan_modes", "npf_run_static", "npf_run_interaction", "npf_taylor_fill",
]
A_DERIVATIVE, A_TAYLOR = 0, 1


class NpfError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: error {code}: {msg}")
        self.code = code


class NpfTensor(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("order", ctypes.c_int32),
        ("values", ctypes.c_void_p), ("col_rank", ctypes.c_void_p),
        ("col_ptr", ctypes.c_void_p), ("row_k", ctypes.c_void_p),
        ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("seed", ctypes.c_uint64), ("scale", ctypes.c_double),
    ]


class NpfPoly(ctypes.Structure):
    _fields_ = [
        ("n_terms", ctypes.c_int64), ("eq_ptr", ctypes.c_void_p), ("coef", ctypes.c_void_p),
        ("var", ctypes.c_void_p), ("max_degree", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("x_eq", ctypes.c_void_p),
    ]


class NpfKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class NpfProblem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("order_max", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("eps", ctypes.c_double), ("tau", ctypes.c_double), ("delta", ctypes.c_double),
        ("hbm_budget_bytes", ctypes.c_int64), ("block_modes", ctypes.c_int64),
        ("flags", ctypes.c_int32), ("support_max", ctypes.c_int32),
        ("a_convention", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("n_modes", ctypes.c_int64), ("modes", ctypes.c_void_p), ("conj_of", ctypes.c_void_p),
        ("host_U", ctypes.c_void_p), ("host_V", ctypes.c_void_p),
        ("host_lambda", ctypes.c_void_p), ("check_tol", ctypes.c_double),
    ]


NPF_FLAG_NO_GRAPH = 1


class NpfPlanReport(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("order_max", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_int64), ("block_modes", ctypes.c_int64),
        ("n_blocks", ctypes.c_int64),
        ("unique_tuples", ctypes.c_int64 * (NPF_MAX_ORDER + 1)),
        ("modal_entries", ctypes.c_int64),
        ("output_modes", ctypes.c_int64), ("computed_modes", ctypes.c_int64),
    ]


class NpfBatchLaunch(ctypes.Structure):
    _fields_ = [("wave", ctypes.c_int32), ("kind", ctypes.c_int32), ("npad", ctypes.c_int32),
                ("order", ctypes.c_int32), ("stage", ctypes.c_int32), ("systems", ctypes.c_int32),
                ("workgroups", ctypes.c_int64), ("flops", ctypes.c_double), ("ms", ctypes.c_double)]


class NpfBatchReport(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("systems", "waves", "workspace_bytes",
                                               "modal_entries", "launches", "shared_launches")]


_lib = None


def lib():
    """Load libnpf.so.  Raises if it is missing: there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2509_08968_amd/build.py "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.npf_plan_create.argtypes = [ctypes.POINTER(NpfProblem), ctypes.POINTER(P)]
        L.npf_plan_info.argtypes = [P, ctypes.POINTER(NpfPlanReport)]
        L.npf_plan_modes.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.npf_plan_destroy.argtypes = [P]
        L.npf_plan_destroy.restype = None
        L.npf_modal_contract.argtypes = [P, i32, i64, ctypes.POINTER(NpfTensor), P, P, P, i64, P, P]
        L.npf_normal_form.argtypes = [P, i32, i64, P, P, P]
        L.npf_assemble.argtypes = [P, i32, i64, P, P, P, P]
        L.npf_finalize.argtypes = [P, P, P, P, P, P]
        L.npf_run.argtypes = [P, ctypes.POINTER(NpfTensor), P, P, P, P, i64, P, P, P]
        L.npf_run_static.argtypes = [P, ctypes.POINTER(NpfTensor), P, P, P, P, P, P]
        L.npf_run_interaction.argtypes = [P, ctypes.POINTER(NpfTensor), P, P, P, P, i64, P, P, P,
                                          P]
        L.npf_alg1_batches.argtypes = [i32, i64, dbl, i32, ctypes.POINTER(i64),
                                       ctypes.POINTER(i64), ctypes.POINTER(dbl),
                                       ctypes.POINTER(dbl)]
        L.npf_alg1_batches.restype = i64
        L.npf_plan_profile.argtypes = [P, i32]
        L.npf_plan_kernel_times.argtypes = [P, ctypes.POINTER(NpfKernelTime), i32,
                                            ctypes.POINTER(i32)]
        L.npf_hash_fill.argtypes = [i64, i32, ctypes.c_uint64, dbl, i64, i64, P, P]
        L.npf_taylor_fill.argtypes = [i64, i32, ctypes.POINTER(NpfPoly), i64, i64, P, P]
        PP = ctypes.POINTER(P)
        L.npf_batch_create.argtypes = [ctypes.POINTER(NpfProblem), i64, i64, ctypes.POINTER(P)]
        L.npf_batch_info.argtypes = [P, ctypes.POINTER(NpfBatchReport)]
        L.npf_batch_destroy.argtypes = [P]
        L.npf_batch_destroy.restype = None
        L.npf_batch_run.argtypes = [P, ctypes.POINTER(NpfTensor), PP, PP, PP, P, i64, PP, PP, P]
        L.npf_batch_tune.argtypes = [P, ctypes.POINTER(NpfTensor), PP, PP, PP, P, i64, PP, PP, P,
                                     ctypes.POINTER(i64)]
        L.npf_batch_time.argtypes = [P, ctypes.POINTER(NpfTensor), PP, PP, PP, P, i64, PP, PP, P]
        L.npf_batch_launches.argtypes = [P, ctypes.POINTER(NpfBatchLaunch), i64, ctypes.POINTER(i64)]
        L.npf_error_string.argtypes = [ctypes.c_int]
        L.npf_error_string.restype = ctypes.c_char_p
        L.npf_last_error.argtypes = []
        L.npf_last_error.restype = ctypes.c_char_p
        for f in ("npf_plan_create", "npf_plan_info", "npf_modal_contract", "npf_normal_form",
                  "npf_assemble", "npf_finalize", "npf_run", "npf_plan_profile",
                  "npf_plan_kernel_times", "npf_hash_fill", "npf_batch_create",
                  "npf_batch_info", "npf_batch_run", "npf_batch_tune", "npf_batch_launches",
                  "npf_batch_time", "npf_plan_modes", "npf_run_static",
                  "npf_run_interaction", "npf_taylor_fill"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != NPF_OK:
        raise NpfError(rc, where, lib().npf_last_error().decode())


def alg1_batches(n_dim: int, n_s: int, m_limit_gb: float, bytes_per_entry: int = 8):
    """Alg. 1 arithmetic (host only): batch count and largest batch per dimension."""
    BC = (ctypes.c_int64 * n_dim)()
    mb = (ctypes.c_int64 * n_dim)()
    tot, per = ctypes.c_double(), ctypes.c_double()
    nb = lib().npf_alg1_batches(n_dim, n_s, m_limit_gb, bytes_per_entry, BC, mb,
                                ctypes.byref(tot), ctypes.byref(per))
    if nb < 0:
        raise ValueError("npf_alg1_batches rejected its arguments")
    return {"batches": int(nb), "BC": list(BC), "max_batch": list(mb),
            "total_gb": tot.value, "batch_gb": per.value}


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def conj_pairs(lam) -> np.ndarray:
    """conj_of for a spectrum whose complex eigenvalues come in exactly conjugate pairs (as
    for a real system): the mode with the conjugate eigenvalue, itself for a real one."""
    lam = np.asarray(lam, np.complex128)
    out = np.arange(len(lam), dtype=np.int64)
    index = {}
    for i, v in enumerate(lam):
        index.setdefault((v.real, v.imag), []).append(i)
    for i, v in enumerate(lam):
        if v.imag != 0:
            cands = index.get((v.real, -v.imag), [])
            if len(cands) != 1 or len(index[(v.real, v.imag)]) != 1:
                raise ValueError(f"mode {i} has no unique conjugate partner")
            out[i] = cands[0]
    return out


class Plan:
    """Owns an npf_plan_t (host metadata only).

    modes: output modes (None = all); conj_of: mode pairing of a real system (conj_pairs);
    taylor: A_M holds Taylor coefficients (no 1/M!); check: (U, V, lam) host arrays for the
    planner's precondition checks (Psi Phi = I, the pairing)."""

    def __init__(self, n: int, order_max: int, precision: str = "fp64", eps: float = 1e-9,
                 tau: float = 1e-2, delta: float = 1.0, budget_bytes: int = 0,
                 block_modes: int = 0, graph: bool = True, support_max: int = 0,
                 modes=None, conj_of=None, taylor: bool = False, check=None,
                 check_tol: float = 0.0):
        keep = []

        def arr(a, dt):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a.ctypes.data_as(ctypes.c_void_p)

        m = None if modes is None else np.asarray(modes, np.int64)
        hu, hv, hl = (None, None, None) if check is None else check
        prob = NpfProblem(n, order_max, PRECISIONS[precision], eps, tau, delta, budget_bytes,
                          block_modes, 0 if graph else NPF_FLAG_NO_GRAPH, int(support_max),
                          A_TAYLOR if taylor else A_DERIVATIVE, 0,
                          0 if m is None else len(m), arr(m, np.int64), arr(conj_of, np.int64),
                          arr(hu, np.complex128), arr(hv, np.complex128), arr(hl, np.complex128),
                          float(check_tol))
        h = ctypes.c_void_p()
        _check(lib().npf_plan_create(ctypes.byref(prob), ctypes.byref(h)), "npf_plan_create")
        self._h = h
        self.n, self.order_max, self.precision = n, order_max, precision
        r = NpfPlanReport()
        _check(lib().npf_plan_info(self._h, ctypes.byref(r)), "npf_plan_info")
        self.workspace_bytes = r.workspace_bytes
        self.block_modes = r.block_modes
        self.n_blocks = r.n_blocks
        self.unique_tuples = list(r.unique_tuples)
        self.modal_entries = r.modal_entries
        self.output_modes = r.output_modes
        self.computed_modes = r.computed_modes

    def modes(self):
        """(computed modes in block order, output mode each fills by conjugation or -1)."""
        nc = self.computed_modes
        c = (ctypes.c_int64 * max(1, nc))()
        f = (ctypes.c_int64 * max(1, nc))()
        _check(lib().npf_plan_modes(self._h, c, f), "npf_plan_modes")
        return list(c)[:nc], list(f)[:nc]

    def close(self):
        if self._h:
            lib().npf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool = True):
        """Record HIP events around every kernel launch of later calls (on their stream)."""
        _check(lib().npf_plan_profile(self._h, 1 if enable else 0), "npf_plan_profile")

    def kernel_times(self):
        """{kernel name: (launches, total ms)} of the recorded launches (waits for them)."""
        cap = 256
        arr = (NpfKernelTime * cap)()
        cnt = ctypes.c_int32()
        _check(lib().npf_plan_kernel_times(self._h, arr, cap, ctypes.byref(cnt)),
               "npf_plan_kernel_times")
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms)
                for i in range(min(cnt.value, cap))}

    def workspace(self, device):
        import torch
        return torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=device)

    def modal_contract(self, order, block, A: "DeviceTensor", U, V, ws, C_out, stream=None):
        _check(lib().npf_modal_contract(self._h, order, block, ctypes.byref(A.desc), _ptr(U),
                                        _ptr(V), _ptr(ws), ws.numel(), _ptr(C_out),
                                        _stream(stream)), "npf_modal_contract")

    def normal_form(self, order, block, lam, C, stream=None):
        _check(lib().npf_normal_form(self._h, order, block, _ptr(lam), _ptr(C), _stream(stream)),
               "npf_normal_form")

    def assemble(self, order, block, h, U, P_acc, stream=None):
        _check(lib().npf_assemble(self._h, order, block, _ptr(h), _ptr(U), _ptr(P_acc),
                                  _stream(stream)), "npf_assemble")

    def finalize(self, U, V, P_sum, npf_out, stream=None):
        _check(lib().npf_finalize(self._h, _ptr(U), _ptr(V), _ptr(P_sum), _ptr(npf_out),
                                  _stream(stream)), "npf_finalize")

    def run_interaction(self, tensors: List["DeviceTensor"], U, V, lam, ws, inpf_out, P_out=None,
                        npf_out=None, stream=None):
        """npf_run_interaction: the NPFs and the interaction factors of eqs. (8)-(9)."""
        arr = (NpfTensor * len(tensors))(*[t.desc for t in tensors])
        _check(lib().npf_run_interaction(self._h, arr, _ptr(U), _ptr(V), _ptr(lam), _ptr(ws),
                                         ws.numel(), _ptr(P_out), _ptr(npf_out), _ptr(inpf_out),
                                         _stream(stream)), "npf_run_interaction")

    def run_static(self, tensors: List["DeviceTensor"], U, V, lam, P_out=None, npf_out=None,
                   stream=None):
        """npf_run_static: the hot path on the library's own static workspace."""
        arr = (NpfTensor * len(tensors))(*[t.desc for t in tensors])
        _check(lib().npf_run_static(self._h, arr, _ptr(U), _ptr(V), _ptr(lam), _ptr(P_out),
                                    _ptr(npf_out), _stream(stream)), "npf_run_static")

    def run(self, tensors: List["DeviceTensor"], U, V, lam, ws, P_out=None, npf_out=None,
            stream=None):
        arr = (NpfTensor * len(tensors))(*[t.desc for t in tensors])
        _check(lib().npf_run(self._h, arr, _ptr(U), _ptr(V), _ptr(lam), _ptr(ws), ws.numel(),
                             _ptr(P_out), _ptr(npf_out), _stream(stream)), "npf_run")


@dataclass
class DeviceTensor:
    """Device copy of one packed derivative tensor and its npf_tensor descriptor."""
    order: int
    kind: int
    tensors: Dict[str, object] = field(default_factory=dict)
    desc: NpfTensor = None


def sparse_columns(A: np.ndarray, support: Optional[np.ndarray] = None):
    """Compress a packed tensor [n, U_M] by sorted tuple: (col_rank, col_ptr, row_k, values)."""
    cols = np.arange(A.shape[1]) if support is None else np.asarray(support, np.int64)
    sub = A[:, cols]
    nz = sub != 0
    keep = nz.any(axis=0)
    cols, sub, nz = cols[keep], sub[:, keep], nz[:, keep]
    counts = nz.sum(axis=0)
    col_ptr = np.zeros(len(cols) + 1, np.int64)
    np.cumsum(counts, out=col_ptr[1:])
    kk, cc = np.nonzero(nz.T)           # column-major walk: by column, then state
    row_k = cc.astype(np.int32)
    values = sub.T[kk, cc].astype(np.float64)
    return cols.astype(np.int64), col_ptr, row_k, values


def _at_least_one(a: np.ndarray) -> np.ndarray:
    return a if a.size else np.zeros(1, a.dtype)


def upload_tensor(A: np.ndarray, order: int, device, sparse: bool = False,
                  support: Optional[np.ndarray] = None) -> DeviceTensor:
    import torch
    if not sparse:
        vals = torch.from_numpy(np.ascontiguousarray(A, np.float64)).to(device)
        desc = NpfTensor(SRC_DENSE, order, vals.data_ptr(), None, None, None, 0, 0)
        return DeviceTensor(order, SRC_DENSE, {"values": vals}, desc)
    cols, ptr, rows, vals = sparse_columns(A, support)
    t = {
        "values": torch.from_numpy(_at_least_one(vals)).to(device),
        "col_rank": torch.from_numpy(_at_least_one(cols)).to(device),
        "col_ptr": torch.from_numpy(ptr).to(device),
        "row_k": torch.from_numpy(_at_least_one(rows)).to(device),
    }
    desc = NpfTensor(SRC_SPARSE, order, t["values"].data_ptr(), t["col_rank"].data_ptr(),
                     t["col_ptr"].data_ptr(), t["row_k"].data_ptr(), len(cols), len(vals))
    return DeviceTensor(order, SRC_SPARSE, t, desc)


def hash_tensor(order: int, seed: int, scale: float) -> DeviceTensor:
    """Descriptor of a hash-generated tensor (generated on the device, nothing stored)."""
    desc = NpfTensor(SRC_HASH, order, None, None, None, None, 0, 0, int(seed), float(scale))
    return DeviceTensor(order, SRC_HASH, {}, desc)


def hash_fill(n: int, order: int, seed: int, scale: float, k0: int, k1: int, out, stream=None):
    """npf_hash_fill: rows [k0, k1) of a hash-generated tensor into the float64 device
    tensor ``out`` (at least (k1 - k0) * binom(n + order - 1, order) elements)."""
    _check(lib().npf_hash_fill(n, order, int(seed), float(scale), k0, k1, _ptr(out),
                               _stream(stream)), "npf_hash_fill")


class DevicePoly:
    """A polynomial vector field in device memory (the npf_poly arrays), from a dict with
    eq_ptr [n+1], coef [T], var [T, D] (padded with -1) and x_eq ([n] or None)."""

    def __init__(self, terms, device):
        import torch
        var = np.ascontiguousarray(terms["var"], np.int32)
        self.n = int(terms["n"])
        self.t = {
            "eq_ptr": torch.from_numpy(np.ascontiguousarray(terms["eq_ptr"], np.int64)).to(device),
            "coef": torch.from_numpy(_at_least_one(np.ascontiguousarray(terms["coef"], np.float64))).to(device),
            "var": torch.from_numpy(_at_least_one(var.reshape(-1))).to(device),
        }
        x_eq = terms.get("x_eq")
        if x_eq is not None:
            self.t["x_eq"] = torch.from_numpy(np.ascontiguousarray(x_eq, np.float64)).to(device)
        self.desc = NpfPoly(len(terms["coef"]), self.t["eq_ptr"].data_ptr(), self.t["coef"].data_ptr(),
                            self.t["var"].data_ptr(), var.shape[1], 0,
                            self.t["x_eq"].data_ptr() if x_eq is not None else None)


def taylor_fill(poly: DevicePoly, order: int, k0: int, k1: int, out, stream=None):
    """npf_taylor_fill: rows [k0, k1) of the order-th derivative tensor of the field at its
    expansion point into the float64 device tensor ``out`` (at least
    (k1 - k0) * binom(n + order - 1, order) elements)."""
    _check(lib().npf_taylor_fill(poly.n, order, ctypes.byref(poly.desc), k0, k1, _ptr(out),
                                 _stream(stream)), "npf_taylor_fill")


def taylor_tensor(poly: DevicePoly, order: int, device="cuda:0", batch_rows: int = 0) -> DeviceTensor:
    """The order-th derivative tensor of the field, filled on the device in batches of
    ``batch_rows`` rows (0 = one batch) as a dense tensor descriptor for the hot path."""
    import torch
    n = poly.n
    UM = math.comb(n + order - 1, order)
    vals = torch.empty(n * UM, dtype=torch.float64, device=device)
    step = batch_rows or n
    for k0 in range(0, n, step):
        k1 = min(n, k0 + step)
        taylor_fill(poly, order, k0, k1, vals[k0 * UM:k1 * UM])
    desc = NpfTensor(SRC_DENSE, order, vals.data_ptr(), None, None, None, 0, 0)
    return DeviceTensor(order, SRC_DENSE, {"values": vals}, desc)


@dataclass
class DeviceSystem:
    n: int
    lam: object
    U: object
    V: object
    tensors: List[DeviceTensor]
    orders: List[int]
    support_max: int = 0


def upload_system(sys, device, sparse: Optional[bool] = None,
                  hash_source: bool = True) -> DeviceSystem:
    """Copy one operating point (inputs.System) to the device.  Hash-generated orders get
    a generator descriptor (nothing is copied) unless ``hash_source`` is False and the
    system holds the materialised tensor."""
    import torch

    def c128(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.complex128)).to(device)

    tens = []
    for M in range(2, sys.order_max + 1):
        A = sys.A.get(M)
        if M in sys.hashed and (A is None or hash_source):
            tens.append(hash_tensor(M, *sys.hashed[M]))
            continue
        if A is None:
            A = np.zeros((sys.n, 1))
            tens.append(upload_tensor(A, M, device, sparse=True, support=np.zeros(0, np.int64)))
            continue
        sp = sparse if sparse is not None else (sys.support.get(M) is not None)
        tens.append(upload_tensor(A, M, device, sparse=sp, support=sys.support.get(M)))
    return DeviceSystem(sys.n, c128(sys.lam), c128(sys.U), c128(sys.V), tens,
                        list(range(2, sys.order_max + 1)), sys.support_max)


def compute(sys, precision: str = "fp64", device="cuda:0", budget_bytes: int = 0,
            block_modes: int = 0, sparse: Optional[bool] = None, graph: bool = True,
            hash_source: bool = True, support_max: Optional[int] = None, modes=None,
            conj: bool = False, taylor: bool = False, fill=None, interaction: bool = False):
    """Run the fused hot path on one system; returns (NPF, {M: P_M}) as numpy arrays.
    support_max (default: the system's own bound, 0 when its tensors are not sent sparse)
    selects the lower-indices-first route for sparse orders.  modes: output modes (None =
    all); conj: compute one mode of each conjugate pair and fill the other; taylor: the
    system's A_M hold Taylor coefficients (NPF_A_TAYLOR).  Rows / columns that are not
    written hold `fill` (default NaN).  interaction: also the interaction factors of
    eqs. (8)-(9), returned third as {M: [n states, n modes]}."""
    import torch
    dev = upload_system(sys, device, sparse, hash_source)
    if support_max is None:
        support_max = sys.support_max if sparse in (None, True) else 0
    plan = Plan(sys.n, sys.order_max, precision, sys.eps, sys.tau, sys.delta, budget_bytes,
                block_modes, graph, support_max, modes=modes,
                conj_of=conj_pairs(sys.lam) if conj else None, taylor=taylor)
    ws = plan.workspace(device)
    n, N = sys.n, sys.order_max
    fv = complex(np.nan, np.nan) if fill is None else fill
    P = torch.full((N - 1, n, n), fv, dtype=torch.complex128, device=device)
    npf = torch.full((n, n), fv, dtype=torch.complex128, device=device)
    if interaction:
        Q = torch.full((N - 1, n, n), fv, dtype=torch.complex128, device=device)
        plan.run_interaction(dev.tensors, dev.U, dev.V, dev.lam, ws, Q, P, npf)
    else:
        plan.run(dev.tensors, dev.U, dev.V, dev.lam, ws, P, npf)
    torch.cuda.synchronize(device)
    Ps = {M: P[M - 2].cpu().numpy() for M in range(2, N + 1)}
    out = npf.cpu().numpy()
    plan.close()
    if interaction:
        return out, Ps, {M: Q[M - 2].cpu().numpy() for M in range(2, N + 1)}
    return out, Ps


# ----------------------------------------------------------------------------- batches
class Batch:
    """npf_batch_*: many systems (split-BF16, N <= 4, n <= 256) through the hot path in one
    call; waves of systems under ``budget_bytes`` of workspace."""

    def __init__(self, systems, budget_bytes: int = 0):
        count = len(systems)
        probs = (NpfProblem * count)()
        for q, sy in enumerate(systems):
            probs[q] = NpfProblem(sy.n, sy.order_max, PRECISIONS["bf16x3"], sy.eps, sy.tau,
                                  sy.delta, 0, 0, 0, int(sy.support_max))
        h = ctypes.c_void_p()
        _check(lib().npf_batch_create(probs, count, int(budget_bytes), ctypes.byref(h)),
               "npf_batch_create")
        self._h = h
        self.count = count
        self.orders = [sy.order_max for sy in systems]
        self.ns = [sy.n for sy in systems]
        r = NpfBatchReport()
        _check(lib().npf_batch_info(self._h, ctypes.byref(r)), "npf_batch_info")
        self.report = {f: int(getattr(r, f)) for f, _ in NpfBatchReport._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().npf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, device):
        import torch
        return torch.empty(max(1, self.report["workspace_bytes"]), dtype=torch.uint8, device=device)

    def _arrays(self, dev_systems, P_outs, npf_outs):
        S = self.count
        A = (NpfTensor * (S * (NPF_MAX_ORDER - 1)))()
        for q, d in enumerate(dev_systems):
            for t in d.tensors:
                A[q * (NPF_MAX_ORDER - 1) + t.order - 2] = t.desc
        arr = lambda xs: (ctypes.c_void_p * S)(*[None if x is None else x.data_ptr() for x in xs])
        U = arr([d.U for d in dev_systems])
        V = arr([d.V for d in dev_systems])
        lam = arr([d.lam for d in dev_systems])
        P = arr(P_outs) if P_outs is not None else None
        N = arr(npf_outs)
        return A, U, V, lam, P, N

    def run(self, dev_systems, ws, P_outs, npf_outs, stream=None):
        A, U, V, lam, P, N = self._arrays(dev_systems, P_outs, npf_outs)
        _check(lib().npf_batch_run(self._h, A, U, V, lam, _ptr(ws), ws.numel(), P, N,
                                   _stream(stream)), "npf_batch_run")

    def tune(self, dev_systems, ws, P_outs, npf_outs, stream=None):
        A, U, V, lam, P, N = self._arrays(dev_systems, P_outs, npf_outs)
        chosen = (ctypes.c_int64 * max(1, self.report["shared_launches"]))()
        _check(lib().npf_batch_tune(self._h, A, U, V, lam, _ptr(ws), ws.numel(), P, N,
                                    _stream(stream), chosen), "npf_batch_tune")
        return list(chosen)[: self.report["shared_launches"]]


    def time_launches(self, dev_systems, ws, P_outs, npf_outs, stream=None):
        """One eager run with events around every shared launch; returns the launch records
        (dicts) with their durations."""
        A, U, V, lam, P, N = self._arrays(dev_systems, P_outs, npf_outs)
        _check(lib().npf_batch_time(self._h, A, U, V, lam, _ptr(ws), ws.numel(), P, N,
                                    _stream(stream)), "npf_batch_time")
        return self.launches()

    def launches(self):
        cnt = ctypes.c_int64()
        _check(lib().npf_batch_launches(self._h, None, 0, ctypes.byref(cnt)), "npf_batch_launches")
        arr = (NpfBatchLaunch * max(1, cnt.value))()
        _check(lib().npf_batch_launches(self._h, arr, cnt.value, ctypes.byref(cnt)),
               "npf_batch_launches")
        return [{f: getattr(arr[i], f) for f, _ in NpfBatchLaunch._fields_} for i in range(cnt.value)]


def compute_batch(systems, device="cuda:0", budget_bytes: int = 0, tune: bool = False,
                  stream=None):
    """Run a batch of systems; returns [(NPF, {M: P_M})] per system as numpy arrays."""
    import torch
    devs = [upload_system(sy, device) for sy in systems]
    b = Batch(systems, budget_bytes)
    ws = b.workspace(device)
    P = [torch.empty((sy.order_max - 1, sy.n, sy.n), dtype=torch.complex128, device=device)
         for sy in systems]
    N = [torch.empty((sy.n, sy.n), dtype=torch.complex128, device=device) for sy in systems]
    if tune:
        b.tune(devs, ws, P, N, stream)
    b.run(devs, ws, P, N, stream)
    torch.cuda.synchronize(device)
    out = [(N[q].cpu().numpy(), {M: P[q][M - 2].cpu().numpy() for M in range(2, sy.order_max + 1)})
           for q, sy in enumerate(systems)]
    b.close()
    return out
