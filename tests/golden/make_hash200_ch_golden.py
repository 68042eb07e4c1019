"""Writes hash200_ch.json: oracle values of the modal coefficients C and the normal-form
coefficients h = C / D (Alg. 2 steps 1-11) on sampled sorted tuples, for the sampled output
modes of the n=200, orders 2-4 hash-generated workload (the modes of hash200_modes.json).
Calls only the CPU oracle and the seeded inputs.

Per order M and sampled mode j: 1024 colex ranks r -- the first and last tuples, and 1022
seeded uniform draws from [0, binom(n+M-1, M)) -- with C_M[j, r] and h_M[j, r].

    python tests/golden/make_hash200_ch_golden.py [nthreads]      (several minutes)
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

import oracle                                    # noqa: E402
from paper_2509_08968_amd import inputs as I     # noqa: E402
from make_hash200_golden import sampled_modes     # noqa: E402

SAMPLES = 1024


def sampled_ranks(n, M):
    UM = math.comb(n + M - 1, M)
    rng = np.random.default_rng(I.BASE_SEED + 40 + M)
    r = rng.integers(0, UM, SAMPLES - 2)
    return np.concatenate([[0, UM - 1], np.sort(r)]).astype(np.int64)


def main():
    nthreads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    s = I.workload_hash200()
    modes = sampled_modes(s)
    out = {"workload": "n200-o4-dense-hash", "n": s.n, "modes": modes, "orders": {}}
    for M in s.orders:
        t0 = time.time()
        ref = oracle.sym(s, M, modes=modes, want_C=True, want_h=True, nthreads=nthreads)
        ranks = sampled_ranks(s.n, M)
        C, h = ref["C"][:, ranks], ref["h"][:, ranks]
        del ref
        out["orders"][str(M)] = {
            "ranks": [int(x) for x in ranks],
            "C": [[[float(z.real), float(z.imag)] for z in row] for row in C],
            "h": [[[float(z.real), float(z.imag)] for z in row] for row in h],
        }
        print(f"order {M}: {time.time() - t0:.1f} s", flush=True)
    with open(os.path.join(HERE, "hash200_ch.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
