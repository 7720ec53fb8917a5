// Host tools of the scheduling study: list scheduling (Step 3 of Algorithm PH, every job to
// the least-loaded machine in a given order) and Kendall's rank correlation with the tie
// correction of the paper's rank-correlation section (the tau_b form).
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <functional>
#include <queue>
#include <utility>
#include <vector>

#include "../../include/hperm.h"

hperm_status hperm_list_schedule(int32_t n, const uint64_t *times, const int32_t *order,
                                 int32_t machines, uint64_t *makespan, uint64_t *loads) {
    if (n < 0 || machines < 1 || !makespan || (n > 0 && (!times || !order))) return HPERM_E_INVALID;
    std::vector<char> seen((size_t)n, 0);
    for (int32_t q = 0; q < n; ++q) {
        const int32_t k = order[q];
        if (k < 0 || k >= n || seen[(size_t)k]) return HPERM_E_INVALID;
        seen[(size_t)k] = 1;
    }
    // min-heap of (load, machine): the least-loaded machine, the lowest index among equals
    using Slot = std::pair<uint64_t, int32_t>;
    std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
    for (int32_t i = 0; i < machines; ++i) heap.push({0, i});
    std::vector<uint64_t> load((size_t)machines, 0);
    for (int32_t q = 0; q < n; ++q) {
        Slot s = heap.top();
        heap.pop();
        s.first += times[order[q]];
        load[(size_t)s.second] = s.first;
        heap.push(s);
    }
    *makespan = *std::max_element(load.begin(), load.end());
    if (loads) std::copy(load.begin(), load.end(), loads);
    return HPERM_OK;
}

namespace {

// Pairs tied within runs of equal values of a sorted sequence: sum of t(t-1)/2.
template <class It, class Eq>
uint64_t tied_pairs(It first, It last, Eq eq) {
    uint64_t total = 0, run = 1;
    for (It it = first; it != last; ++it) {
        if (it != first && eq(*(it - 1), *it)) {
            ++run;
        } else {
            total += run * (run - 1) / 2;
            run = 1;
        }
    }
    return total + run * (run - 1) / 2;
}

// Merge sort of v by value, returning the number of pairs (i < j) with v[i] > v[j]
// (strict inversions; equal values are not counted).
uint64_t sort_count_inversions(std::vector<double> &v) {
    const size_t n = v.size();
    std::vector<double> tmp(n);
    uint64_t inv = 0;
    for (size_t width = 1; width < n; width *= 2) {
        for (size_t lo = 0; lo < n; lo += 2 * width) {
            const size_t mid = std::min(lo + width, n), hi = std::min(lo + 2 * width, n);
            size_t i = lo, j = mid, k = lo;
            while (i < mid && j < hi) {
                if (v[j] < v[i]) {   // v[j] jumps every remaining left element
                    inv += mid - i;
                    tmp[k++] = v[j++];
                } else {
                    tmp[k++] = v[i++];
                }
            }
            while (i < mid) tmp[k++] = v[i++];
            while (j < hi) tmp[k++] = v[j++];
        }
        v.swap(tmp);
    }
    return inv;
}

}  // namespace

hperm_status hperm_kendall_tau(int32_t n, const double *x, const double *y, double *tau,
                               double *z, double *p) {
    if (n < 2 || !x || !y || !tau) return HPERM_E_INVALID;
    for (int32_t i = 0; i < n; ++i)
        if (isnan(x[i]) || isnan(y[i])) return HPERM_E_INVALID;
    // sort by (x, y): pairs tied in x (T), tied in both; then the discordant pairs are the
    // strict inversions of y in that order (Knight's O(n log n) method)
    std::vector<std::pair<double, double>> xy((size_t)n);
    for (int32_t i = 0; i < n; ++i) xy[(size_t)i] = {x[i], y[i]};
    std::sort(xy.begin(), xy.end());
    const uint64_t n0 = (uint64_t)n * (uint64_t)(n - 1) / 2;
    const uint64_t t_x = tied_pairs(xy.begin(), xy.end(), [](const auto &a, const auto &b) { return a.first == b.first; });
    const uint64_t t_xy = tied_pairs(xy.begin(), xy.end(), [](const auto &a, const auto &b) { return a == b; });
    std::vector<double> ys((size_t)n);
    for (int32_t i = 0; i < n; ++i) ys[(size_t)i] = xy[(size_t)i].second;
    const uint64_t disc = sort_count_inversions(ys);   // leaves ys sorted
    const uint64_t t_y = tied_pairs(ys.begin(), ys.end(), [](double a, double b) { return a == b; });
    if (t_x == n0 || t_y == n0) return HPERM_E_INVALID;
    // pairs untied in both: concordant + discordant = n0 - t_x - t_y + t_xy
    const double untied = (double)n0 - (double)t_x - (double)t_y + (double)t_xy;
    const double s = untied - 2.0 * (double)disc;   // concordant - discordant
    *tau = s / sqrt((double)(n0 - t_x) * (double)(n0 - t_y));
    const double var = 2.0 * (2.0 * n + 5.0) / (9.0 * n * (n - 1.0));
    const double zz = *tau / sqrt(var);
    if (z) *z = zz;
    if (p) *p = erfc(fabs(zz) / sqrt(2.0));
    return HPERM_OK;
}
