"""The scheduling study (Step 3 of Algorithm PH and the rank-correlation analysis of the
paper's load-balancing section): the oracle against textbook facts, then the library's native
list scheduling and Kendall's tau against the oracle."""
import itertools
import math

import numpy as np
import pytest

from oracle import efficiency, kendall_tau, list_schedule, opt_makespan_brute


@pytest.fixture(scope="module")
def hperm():
    """The library's host-side calls (no GPU needed for these)."""
    import paper_1112_6072_amd as hp
    return hp


def lpt_order(times):
    """Non-increasing times, ties in index order (a stable sort)."""
    return sorted(range(len(times)), key=lambda k: -int(times[k]))


# ------------------------------------------------------------------ oracle pins
@pytest.mark.parametrize("k", [2, 3, 4])
def test_graham_lpt_worst_case(k):
    """Graham's instance: 2k+1 jobs of lengths 2k-1, 2k-1, 2k-2, 2k-2, ..., k+1, k+1, k, k, k on
    k machines; LPT gives 4k-1 while the optimum is 3k, the 4/3 - 1/(3k) bound with equality."""
    times = [t for t in range(2 * k - 1, k, -1) for _ in range(2)] + [k, k, k]
    assert len(times) == 2 * k + 1
    ms, loads = list_schedule(times, lpt_order(times), k)
    assert ms == 4 * k - 1
    assert sum(loads) == sum(times)
    assert opt_makespan_brute(times, k) == 3 * k
    assert ms / (3 * k) == pytest.approx(4 / 3 - 1 / (3 * k))


@pytest.mark.parametrize("k", [2, 3, 5])
def test_list_scheduling_worst_case(k):
    """k(k-1) unit jobs, then one job of length k: list scheduling ends at 2k-1, the optimum is
    k: the 2 - 1/k bound with equality; LPT order finds the optimum."""
    times = [1] * (k * (k - 1)) + [k]
    ms, _ = list_schedule(times, list(range(len(times))), k)
    assert ms == 2 * k - 1
    assert list_schedule(times, lpt_order(times), k)[0] == k
    assert efficiency(times, k, k) == 1.0


def test_list_scheduling_bounds_random():
    """On random small instances: LS <= (2 - 1/k) OPT for any order, LPT <= (4/3 - 1/(3k)) OPT."""
    rng = np.random.default_rng(5)
    for _ in range(60):
        k = int(rng.integers(2, 4))
        times = [int(t) for t in rng.integers(1, 20, int(rng.integers(k, 8)))]
        opt = opt_makespan_brute(times, k)
        order = list(rng.permutation(len(times)))
        assert list_schedule(times, order, k)[0] <= (2 - 1 / k) * opt + 1e-9
        assert list_schedule(times, lpt_order(times), k)[0] <= (4 / 3 - 1 / (3 * k)) * opt + 1e-9
        assert opt >= max(max(times), math.ceil(sum(times) / k))


def test_kendall_hand_example_with_ties():
    """x = (1, 2, 2, 3), y = (1, 3, 2, 4): five concordant pairs, one pair tied in x, so
    S = 5, T = 1, U = 0 and tau = 5 / sqrt(5 * 6)."""
    tau, _, _ = kendall_tau([1, 2, 2, 3], [1, 3, 2, 4])
    assert tau == pytest.approx(5 / math.sqrt(30), rel=1e-15)
    assert kendall_tau([1, 2, 3, 4, 5], [2, 4, 6, 8, 10])[0] == 1.0
    assert kendall_tau([1, 2, 3, 4, 5], [5, 4, 3, 2, 1])[0] == -1.0


def test_kendall_null_distribution_exact():
    """Over all 5! orders of y against x = (1..5) (no ties), tau has mean 0 and variance
    exactly 2(2n+5) / (9n(n-1)) = 1/6, the variance the paper quotes."""
    n = 5
    taus = [kendall_tau(list(range(n)), list(p))[0] for p in itertools.permutations(range(n))]
    assert sum(taus) == pytest.approx(0.0, abs=1e-12)
    var = sum(t * t for t in taus) / len(taus)
    assert var == pytest.approx(2 * (2 * n + 5) / (9 * n * (n - 1)), rel=1e-12)
    assert var == pytest.approx(1 / 6, rel=1e-12)


def test_kendall_matches_an_independent_library():
    """scipy's tau_b (Knight's algorithm) agrees with the pairwise definition, ties included."""
    from scipy.stats import kendalltau
    rng = np.random.default_rng(9)
    for n in (7, 50, 400):
        x = rng.integers(0, 6, n).astype(float)
        y = x + rng.integers(0, 4, n)
        assert kendall_tau(x, y)[0] == pytest.approx(kendalltau(x, y).statistic, abs=1e-12)


# ------------------------------------------------------------------ library against the oracle
def test_native_list_schedule_matches_oracle(hperm):
    rng = np.random.default_rng(21)
    for n in (0, 1, 5, 64, 1000):
        times = rng.integers(1, 10 ** 12, n, dtype=np.int64).astype(np.uint64)
        times[: n // 3] = times[0] if n else 0   # equal times exercise the tie rule
        for k in (1, 2, 3, 7, 32):
            for order in (np.arange(n), rng.permutation(n), np.array(lpt_order(list(times)), dtype=np.int64)):
                ms, loads = hperm.list_schedule(times, order, k)
                ms_o, loads_o = list_schedule([int(t) for t in times], list(order), k)
                assert ms == ms_o
                assert [int(v) for v in loads] == loads_o


def test_native_kendall_matches_oracle(hperm):
    rng = np.random.default_rng(22)
    for n in (2, 3, 10, 300, 2500):
        x = rng.integers(0, max(2, n // 4), n).astype(float)
        y = 0.5 * x + rng.normal(size=n).round(1)
        tau, z, p = hperm.kendall_tau(x, y)
        tau_o, z_o, p_o = kendall_tau(x, y)
        assert tau == pytest.approx(tau_o, abs=1e-12)
        assert z == pytest.approx(z_o, rel=1e-12, abs=1e-12)
        assert p == pytest.approx(p_o, rel=1e-9, abs=1e-300)


def test_native_schedule_rejects_bad_input(hperm):
    with pytest.raises(hperm.HpermError):
        hperm.list_schedule([1, 2, 3], [0, 0, 1], 2)
    with pytest.raises(hperm.HpermError):
        hperm.list_schedule([1, 2, 3], [0, 1, 2], 0)
    with pytest.raises(hperm.HpermError):
        hperm.kendall_tau([1.0], [2.0])
    with pytest.raises(hperm.HpermError):
        hperm.kendall_tau([1.0, 1.0, 1.0], [1.0, 2.0, 3.0])
    with pytest.raises(hperm.HpermError):
        hperm.kendall_tau([1.0, float("nan")], [1.0, 2.0])
