"""Writes example2_oracle.txt: the FP64 oracle's TT-UTV of the Example 2
tensor (Sec. 4.1: B = sin(sqrt(sum_k ((i_k-1)/(I-1))^2)), I = 160, d = 4) at
the prescribed accuracies of Table "Beps", for TT-URV right to left (Alg. 3,
prescribed-accuracy form) and TT-ULV left to right (Alg. 2), q = 1, p = 8,
seed 2: ranks, relative error of the reconstruction and the reported bound.
Calls only the oracle and the input generator; about ten minutes on 8 cores.

    python tests/golden/make_example2_oracle.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import ttgen  # noqa: E402

EPS = (1e-2, 1e-3, 1e-4, 1e-5)
FORMS = (("R2L", "URV"), ("L2R", "ULV"))
OPTS = dict(q=1, p=8, seed=2)


def main():
    a = ttgen.sin_norm_tensor(4, 160)
    norm = float(np.linalg.norm(a))
    lines = ["# Example 2 (Sec. 4.1), 160^4 FP64, TT-UTV by the FP64 oracle, q=1, p=8, seed=2",
             "# written by tests/golden/make_example2_oracle.py",
             "# eps sweep variant r1 r2 r3 rse err_bound_rel"]
    for eps in EPS:
        for sweep, variant in FORMS:
            cores, rep = oracle.tt_utv(a, [160] * 4, eps=eps, sweep=sweep, variant=variant, **OPTS)
            rse = float(np.linalg.norm(oracle.tt_reconstruct(cores) - a)) / norm
            r = rep["ranks"]
            lines.append(f"{eps:g} {sweep} {variant} {r[1]} {r[2]} {r[3]} {rse:.6e} {rep['err_bound'] / rep['norm_A']:.6e}")
            print(lines[-1], flush=True)
    with open(os.path.join(HERE, "example2_oracle.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
