// Host tools of the scheduling study: list scheduling (Step 3 of Algorithm PH, every job to
// the least-loaded machine in a given order), Kendall's rank correlation with the tie
// correction of the paper's rank-correlation section (the tau_b form), and the linear
// regression of Section 3.1 (eqs. 4-6): least squares with the printed R^2, stepwise
// selection, and the matrix invariants it regresses on.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
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

// ---- the regression of the paper's Section 3.1 (eqs. 4-6) --------------------------------

namespace {

// Least squares of y on the chosen columns of X (row-major n x k) with an intercept, by
// modified Gram-Schmidt on the centred and scaled columns in long double. coef (may be NULL)
// receives a0 and one coefficient per chosen column (in X's units); returns the residual sum
// of squares, or -1 when the chosen columns are linearly dependent (or n too small).
long double fit(int32_t n, int32_t k, const double *X, const double *y, const std::vector<int32_t> &cols,
                double *coef, double *r2) {
    const size_t c = cols.size();
    if ((size_t)n < c + 2) return -1.0L;
    long double ybar = 0;
    for (int32_t i = 0; i < n; ++i) ybar += y[i];
    ybar /= n;
    std::vector<long double> mean(c, 0), scale(c, 0), q((size_t)n * c), r(c * c, 0), b(c, 0);
    for (size_t j = 0; j < c; ++j) {
        for (int32_t i = 0; i < n; ++i) mean[j] += X[(size_t)i * k + cols[j]];
        mean[j] /= n;
        for (int32_t i = 0; i < n; ++i) {
            const long double v = X[(size_t)i * k + cols[j]] - mean[j];
            q[(size_t)i * c + j] = v;
            scale[j] += v * v;
        }
        scale[j] = sqrtl(scale[j]);
        if (!(scale[j] > 0)) return -1.0L;   // a constant column
        for (int32_t i = 0; i < n; ++i) q[(size_t)i * c + j] /= scale[j];
    }
    // Q R = the centred, scaled columns
    for (size_t j = 0; j < c; ++j) {
        for (size_t l = 0; l < j; ++l) {
            long double d = 0;
            for (int32_t i = 0; i < n; ++i) d += q[(size_t)i * c + l] * q[(size_t)i * c + j];
            r[l * c + j] = d;
            for (int32_t i = 0; i < n; ++i) q[(size_t)i * c + j] -= d * q[(size_t)i * c + l];
        }
        long double nrm = 0;
        for (int32_t i = 0; i < n; ++i) nrm += q[(size_t)i * c + j] * q[(size_t)i * c + j];
        nrm = sqrtl(nrm);
        if (!(nrm > 1e-12L)) return -1.0L;
        r[j * c + j] = nrm;
        for (int32_t i = 0; i < n; ++i) q[(size_t)i * c + j] /= nrm;
    }
    // R b = Q^T (y - ybar)
    std::vector<long double> qty(c, 0);
    for (size_t j = 0; j < c; ++j)
        for (int32_t i = 0; i < n; ++i) qty[j] += q[(size_t)i * c + j] * (y[i] - ybar);
    for (size_t j = c; j-- > 0;) {
        long double v = qty[j];
        for (size_t l = j + 1; l < c; ++l) v -= r[j * c + l] * b[l];
        b[j] = v / r[j * c + j];
    }
    long double rss = 0, ssr = 0, sst = 0, a0 = ybar;
    for (size_t j = 0; j < c; ++j) a0 -= b[j] / scale[j] * mean[j];
    for (int32_t i = 0; i < n; ++i) {
        long double yh = a0;
        for (size_t j = 0; j < c; ++j) yh += b[j] / scale[j] * X[(size_t)i * k + cols[j]];
        rss += (y[i] - yh) * (y[i] - yh);
        ssr += (yh - ybar) * (yh - ybar);
        sst += (y[i] - ybar) * (y[i] - ybar);
    }
    if (coef) {
        coef[0] = (double)a0;
        for (size_t j = 0; j < c; ++j) coef[j + 1] = (double)(b[j] / scale[j]);
    }
    if (r2) *r2 = sst > 0 ? (double)(ssr / sst) : 0.0;
    return rss;
}

bool finite_all(int32_t n, int32_t k, const double *X, const double *y) {
    for (size_t e = 0; e < (size_t)n * k; ++e)
        if (!std::isfinite(X[e])) return false;
    for (int32_t i = 0; i < n; ++i)
        if (!std::isfinite(y[i])) return false;
    return true;
}

}  // namespace

hperm_status hperm_ols(int32_t n, int32_t k, const double *X, const double *y, double *coef, double *r2) {
    if (n < 1 || k < 0 || k > 64 || !y || (k > 0 && !X) || !coef || !r2) return HPERM_E_INVALID;
    if (!finite_all(n, k, X, y)) return HPERM_E_INVALID;
    std::vector<int32_t> cols((size_t)k);
    for (int32_t j = 0; j < k; ++j) cols[(size_t)j] = j;
    return fit(n, k, X, y, cols, coef, r2) < 0 ? HPERM_E_INVALID : HPERM_OK;
}

hperm_status hperm_stepwise(int32_t n, int32_t k, const double *X, const double *y, double f_enter,
                            double f_remove, int32_t *chosen, int32_t *n_chosen) {
    if (n < 1 || k < 1 || k > 64 || !X || !y || !chosen || !n_chosen || !(f_enter > 0) || !(f_remove >= 0) ||
        f_remove > f_enter)
        return HPERM_E_INVALID;
    if (!finite_all(n, k, X, y)) return HPERM_E_INVALID;
    std::vector<int32_t> model;
    auto rss_of = [&](const std::vector<int32_t> &m) -> long double {
        if (m.empty()) {
            long double ybar = 0, s = 0;
            for (int32_t i = 0; i < n; ++i) ybar += y[i];
            ybar /= n;
            for (int32_t i = 0; i < n; ++i) s += (y[i] - ybar) * (y[i] - ybar);
            return s;
        }
        return fit(n, k, X, y, m, nullptr, nullptr);
    };
    for (int32_t pass = 0; pass < 4 * k; ++pass) {
        const long double rss = rss_of(model);
        int32_t best = -1;
        long double best_f = f_enter;
        for (int32_t j = 0; j < k; ++j) {
            if (std::find(model.begin(), model.end(), j) != model.end() || n - (int32_t)model.size() - 2 <= 0) continue;
            std::vector<int32_t> m = model;
            m.push_back(j);
            const long double r = rss_of(m);
            if (r < 0) continue;   // dependent on the model's columns: cannot enter
            const long double f = r <= 0 ? INFINITY : (rss - r) / (r / (n - (int32_t)model.size() - 2));
            if (f > best_f) {
                best = j;
                best_f = f;
            }
        }
        if (best < 0) break;
        model.push_back(best);
        while (model.size() > 1) {
            const long double r = rss_of(model);
            int32_t worst = -1;
            long double worst_f = f_remove;
            for (int32_t j : model) {
                std::vector<int32_t> rest;
                for (int32_t c : model)
                    if (c != j) rest.push_back(c);
                const long double f = r <= 0 ? INFINITY : (rss_of(rest) - r) / (r / (n - (int32_t)model.size() - 1));
                if (f < worst_f) {
                    worst = j;
                    worst_f = f;
                }
            }
            if (worst < 0) break;
            model.erase(std::find(model.begin(), model.end(), worst));
        }
    }
    *n_chosen = (int32_t)model.size();
    std::copy(model.begin(), model.end(), chosen);
    return HPERM_OK;
}

hperm_status hperm_matrix_invariants(int32_t m, const uint32_t *a, double *out) {
    if (m < 1 || m > 128 || !a || !out) return HPERM_E_INVALID;
    // |det| by Gaussian elimination with partial pivoting in long double (a float value: the
    // regression's input, not an exact determinant)
    std::vector<long double> w((size_t)m * m);
    for (size_t e = 0; e < (size_t)m * m; ++e) w[e] = a[e];
    long double det = 1;
    for (int32_t c = 0; c < m && det != 0; ++c) {
        int32_t piv = c;
        for (int32_t r = c + 1; r < m; ++r)
            if (fabsl(w[(size_t)r * m + c]) > fabsl(w[(size_t)piv * m + c])) piv = r;
        if (w[(size_t)piv * m + c] == 0) {
            det = 0;
            break;
        }
        if (piv != c)
            for (int32_t j = 0; j < m; ++j) std::swap(w[(size_t)piv * m + j], w[(size_t)c * m + j]);
        det *= w[(size_t)c * m + c];
        for (int32_t r = c + 1; r < m; ++r) {
            const long double f = w[(size_t)r * m + c] / w[(size_t)c * m + c];
            if (f != 0)
                for (int32_t j = c; j < m; ++j) w[(size_t)r * m + j] -= f * w[(size_t)c * m + j];
        }
    }
    long double nnz = 0, rmean = 0, cmean = 0, rvar = 0, cvar = 0;
    std::vector<long double> rs((size_t)m, 0), cs((size_t)m, 0);
    for (int32_t i = 0; i < m; ++i)
        for (int32_t j = 0; j < m; ++j) {
            const uint32_t v = a[(size_t)i * m + j];
            nnz += v != 0;
            rs[(size_t)i] += v;
            cs[(size_t)j] += v;
        }
    for (int32_t i = 0; i < m; ++i) {
        rmean += rs[(size_t)i];
        cmean += cs[(size_t)i];
    }
    rmean /= m;
    cmean /= m;
    for (int32_t i = 0; i < m; ++i) {
        rvar += (rs[(size_t)i] - rmean) * (rs[(size_t)i] - rmean);
        cvar += (cs[(size_t)i] - cmean) * (cs[(size_t)i] - cmean);
    }
    out[0] = (double)fabsl(det);
    out[1] = (double)nnz;
    out[2] = (double)(rvar / m);
    out[3] = (double)(cvar / m);
    return HPERM_OK;
}
