"""CPU oracle for the exact sparse permanent and the KKLLL estimate.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link or run
anything in this package: only the tests, the smoke check and the benchmark's CPU
baseline use it. It shares no code with the GPU library.

Contents
--------
permanent.py   exact per(A) in Python integers: the defining sum over permutations
               (eq. 1), Ryser's inclusion-exclusion, the doubled Nijenhuis-Wilf sum, the
               paper's row/column expansion (eq. 2) and Algorithm H_per (Section 2.1),
               and an independent frontier dynamic programme for large sparse inputs.
kkl.py         the KKLLL estimator (Section 2.3): one trial |det B|^2 for given cube-root
               exponents, the SplitMix64 counter generator that draws them, and the
               log-mean key used to order jobs.
ryser_c.c      plain Ryser in C with 128-bit wrap-around integers, threaded over a list
               of matrices; used only to time a CPU baseline.
schedule.py    the scheduling study (Sections 3.2-3.3): list scheduling to the least-loaded
               processor (Step 3 of Algorithm PH), brute-force optimal makespans, and
               Kendall's tau with the paper's tie correction.
regression.py  the regression of Section 3.1 (eqs. 4-6): exact |det| by fraction-free
               elimination, the five matrix invariants, least squares with the printed R^2,
               and stepwise selection.
"""
from .permanent import (per_brute, per_ryser, nw_doubled_sum, per_nw, e2_children, expand_leaves,
                        choose_line, per_hybrid, per_dp, per_auto)
from .kkl import splitmix64, kkl_exponent, kkl_trial, kkl_key
from .schedule import list_schedule, efficiency, kendall_tau, opt_makespan_brute
from .regression import determinant_abs, invariants, ols, r_squared, stepwise

__all__ = [
    "per_brute", "per_ryser", "nw_doubled_sum", "per_nw", "e2_children", "expand_leaves", "choose_line",
    "per_hybrid", "per_dp", "per_auto", "splitmix64", "kkl_exponent", "kkl_trial", "kkl_key",
    "list_schedule", "efficiency", "kendall_tau", "opt_makespan_brute",
    "determinant_abs", "invariants", "ols", "r_squared", "stepwise",
]
