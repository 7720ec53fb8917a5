"""Write tests/golden/c60_permanental_polynomial.json: the exact coefficients of per(xI - A) for
the truncated icosahedron C60 (the paper's application; its adjacency from the appendix list).

Calls only the oracle: per(xI - A) at x = 0..60 by the frontier dynamic programme (signed
entries), evaluated in parallel processes, then Lagrange interpolation in exact rationals
(oracle.polynomial.interpolate). Run: python tests/golden/make_c60_polynomial.py
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle.permanent import per_dp  # noqa: E402
from oracle.polynomial import interpolate  # noqa: E402


def c60() -> np.ndarray:
    return W.adjacency_matrix(W.read_appendix_adjacency("c60")).astype(np.int64)


def value_at(x: int) -> int:
    """per(xI - A) of C60."""
    M = -c60()
    for i in range(M.shape[0]):
        M[i, i] += x
    return per_dp(M.tolist())


def main():
    t0 = time.time()
    xs = list(range(61))
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        ys = list(ex.map(value_at, xs))
    coeffs = interpolate(ys)
    assert len(coeffs) == 61 and coeffs[60] == 1 and coeffs[59] == 0 and coeffs[58] == 90
    out = {"_comment": "coefficients c_0..c_60 (c_k of x^k) of per(xI - A) for the truncated icosahedron "
                       "(appendix adjacency), from the oracle's frontier DP at x = 0..60 and exact interpolation",
           "coefficients": [str(c) for c in coeffs]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c60_permanental_polynomial.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path, f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
