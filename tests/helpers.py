"""Shared test helpers: error norms and the systems the parity tests run on."""
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
