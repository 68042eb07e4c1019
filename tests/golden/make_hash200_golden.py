"""Writes hash200_modes.json: oracle values for sampled output modes of the n=200,
orders 2-4 hash-generated workload (A_4 alone would be 110 GB in FP64, so the oracle
generates every entry on the fly).  Calls only the CPU oracle and the seeded inputs.

Stored per sampled mode j: the rows P_M[j, :] for M = 2, 3, 4 (eq. (7) reduction of
Alg. 2 steps 12-19) and the NPF column NPF[:, j] (step 20).  The modes are three seeded
draws plus the mode with the smallest order-2 divisor |lam_p + lam_q - lam_j|.

    python tests/golden/make_hash200_golden.py [nthreads]      (several minutes)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle                                    # noqa: E402
from paper_2509_08968_amd import inputs as I     # noqa: E402


def sampled_modes(s):
    rng = np.random.default_rng(I.BASE_SEED + 4 + 1000)
    picks = set(int(x) for x in rng.choice(s.n, 3, replace=False))
    lam = s.lam
    d2 = np.abs(lam[None, :, None] + lam[None, None, :] - lam[:, None, None]).reshape(s.n, -1)
    picks.add(int(np.argmin(d2.min(1))))
    return sorted(picks)


def main():
    nthreads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    s = I.workload_hash200()
    modes = sampled_modes(s)
    out = {"workload": "n200-o4-dense-hash", "n": s.n, "orders": s.orders, "modes": modes,
           "hashed": {str(M): [int(v[0]), float(v[1])] for M, v in s.hashed.items()},
           "P": {}, "npf_columns": None}
    Psum = np.zeros((s.n, s.n), np.complex128)
    for M in s.orders:
        t0 = time.time()
        P = oracle.sym(s, M, modes=modes, nthreads=nthreads)["P"]
        print(f"order {M}: {time.time() - t0:.1f} s", flush=True)
        out["P"][str(M)] = [[[float(z.real), float(z.imag)] for z in row] for row in P]
        Psum[modes] += P
    npf = oracle.assemble(s, Psum)
    out["npf_columns"] = [[[float(z.real), float(z.imag)] for z in npf[:, j]] for j in modes]
    with open(os.path.join(HERE, "hash200_modes.json"), "w") as f:
        json.dump(out, f)
    print("modes", modes)


if __name__ == "__main__":
    main()
