"""Shared test helpers: error norms and the systems the parity tests run on."""
import json
import os

import numpy as np

from paper_2509_08968_amd import inputs as I


def rel(a, b):
    """Relative Frobenius error ||a - b|| / ||b||."""
    a, b = np.asarray(a), np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


# name -> builder of a small system that the oracle finishes in well under a second
PARITY_CASES = {
    "n10-o2-dense": I.workload_small,
    "n12-o3-dense": lambda: I.dense_system(12, [2, 3], 3101),
    "n9-o4-dense-odd": lambda: I.dense_system(9, [2, 3, 4], 3102),
    "n24-o3-blocksparse": lambda: I.block_sparse_system(24, [2, 3], 3103),
    "n37-o2-dense-odd": lambda: I.dense_system(37, [2], 3104),
    "n20-o3-resonant": lambda: I.resonant_system(20, [2, 3], 3105, n_res2=1, n_res3=1),
    "n1-o2": lambda: I.dense_system(1, [2], 3106),
    "n72-o3-dense": lambda: I.dense_system(72, [2, 3], 3107),
    "n130-o2-dense": lambda: I.dense_system(130, [2], 3108),
}

# Plans beyond four orders (the largest order the API accepts is six).
HIGH_ORDER_CASES = {
    "n18-o5-dense": lambda: I.dense_system(18, [2, 3, 4, 5], 3109),
    "n11-o6-dense": lambda: I.dense_system(11, [2, 3, 4, 5, 6], 3110),
}


def mode_errors(got, ref):
    """Errors of a result whose rows are output modes (P_M rows, C/h rows, or NPF columns
    passed transposed): the relative Frobenius error of every row against its own norm, their
    maximum, the pooled relative error and the max-entry error max|got - ref| / max|ref|.
    A row whose reference is exactly zero must be exactly zero (its error is 0 or inf)."""
    a = np.atleast_2d(np.asarray(got))
    b = np.atleast_2d(np.asarray(ref))
    assert a.shape == b.shape, (a.shape, b.shape)
    d = np.linalg.norm(a - b, axis=1)
    nb = np.linalg.norm(b, axis=1)
    per = np.where(nb > 0, d / np.where(nb > 0, nb, 1.0), np.where(d > 0, np.inf, 0.0))
    mb = np.abs(b).max() if b.size else 0.0
    return {"per_mode": per, "per_mode_max": float(per.max()) if per.size else 0.0,
            "pooled": float(rel(a, b)),
            "max_entry": float(np.abs(a - b).max() / mb) if mb > 0 else float(np.abs(a).max())}


# Per-mode guard of the mixed paths, relative to each output mode's own row norm.  The
# stated 1e-6 bound is relative to the norm of the whole quantity (pooled over the modes
# compared); a row whose reduction cancels more than most (sum of |terms| / |P_j| of about
# 4e3 against 150-350 for typical rows, seen at 160 states) has a larger error relative to
# its own small norm -- rounding C once to FP32 already gives 3e-7 there -- so each row
# is held to five times the bound, which still exposes any wrong mode by orders of magnitude.
MODE_GUARD = 5.0


def check(got, ref, tol, what=""):
    """Assert the error of a result whose rows are output modes: pooled over the rows within
    tol, and every row within tol relative to its own norm (MODE_GUARD * tol for the mixed
    paths' bounds, tol >= 1e-8); prints the per-mode, pooled and max-entry errors."""
    e = mode_errors(got, ref)
    worst = int(np.argmax(e["per_mode"])) if e["per_mode"].size else -1
    mode_tol = tol if tol < 1e-8 else MODE_GUARD * tol
    print(f"  {what}: per-mode max {e['per_mode_max']:.2e} (row {worst}), pooled "
          f"{e['pooled']:.2e}, max-entry {e['max_entry']:.2e}", flush=True)
    log = os.environ.get("NPF_PARITY_LOG")
    if log:
        with open(log, "a") as f:
            f.write(json.dumps({"test": os.environ.get("PYTEST_CURRENT_TEST", ""), "what": what,
                                "tol": tol, "per_mode_max": e["per_mode_max"], "worst_row": worst,
                                "pooled": e["pooled"], "max_entry": e["max_entry"]}) + "\n")
    assert e["pooled"] <= tol, (what, "pooled", e["pooled"])
    assert e["per_mode_max"] <= mode_tol, (what, worst, e["per_mode_max"])
    return e
