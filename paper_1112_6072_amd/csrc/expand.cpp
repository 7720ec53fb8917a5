// Host expansion of per(A) into sub-matrix jobs, following expansion (2) and Algorithm
// H_per (Section 2.1) and the pre-expansion of Algorithm PH (Section 2.2).
//
// A node is a sparse matrix of order m (rows as sorted column lists). At each node, s is
// the smallest number of nonzeros in a row or a column (Step 1 of H_per; ties: rows
// first, then the lowest index). s = 0 means per = 0 and the node is dropped. The node
// becomes a job when m <= m_cut, or when s >= s_leaf and m <= m_cap (H_per hands a node
// with s >= 5 to R-NW). Otherwise it is split by expansion (2) along that line: its
// nonzeros v1, v2, ... (increasing column) are taken in pairs, the pair at columns p, q
// giving the child with the row deleted and columns p, q replaced by v_p*y_q + v_q*y_p
// (the first two terms of (2)); repeating (2) on the remainder term A3 consumes the row, so
// k nonzeros give ceil(k/2) children of order m-1. An odd last nonzero is paired with a
// column whose coefficient is 0 (a zero of the row if there is one), i.e. the Laplace term
// v_p * per(minor) with the partner column scaled by v_p. A column line is expanded by the
// same rule on the transpose (rows p, q merged, the column deleted), written directly on
// the row lists.
//
// Jobs are emitted in depth-first order of the expansion tree (the "natural order" of
// Step 3 of Algorithm PH). The top of the tree is split breadth-first into independent
// subtrees that worker threads expand; their job lists are concatenated in subtree order,
// so the result does not depend on the thread count.
#include "expand.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

namespace hp {

namespace {

struct Node {
    int m = 0;
    int nnz = 0;
    std::vector<int32_t> rp;    // m + 1
    std::vector<uint8_t> ci;    // nnz, sorted within a row
    std::vector<uint32_t> v;    // nnz, all nonzero
    void reserve(int n, int nz) {
        rp.resize(n + 1);
        ci.resize(std::max(nz, 1));
        v.resize(std::max(nz, 1));
    }
};

struct RangeError {
    std::string msg;
};

struct LimitError {};   // the job table outgrew ExpandParams::max_bytes

// Proven log2 upper bound of per(B) for a non-negative integer matrix: min of the product
// of row sums and the product of column sums; for a 0-1 matrix also Bregman's bound
// prod_i (r_i!)^(1/r_i) (rows, and columns by transposition).
// log2(k!) / k for k = 0..HP_MAX_N (Bregman's factor of a line with k ones; entry 0 unused).
static const double *bregman_table() {
    static const struct Table {
        double v[HP_MAX_N + 1];
        Table() {
            v[0] = 0.0;
            for (int k = 1; k <= HP_MAX_N; ++k) v[k] = std::lgamma(k + 1.0) / std::log(2.0) / k;
        }
    } t;
    return t.v;
}

// log2(x) of a positive integer-valued line sum: a table below 4096 (the values std::log2
// gives), std::log2 above.
static inline double log2_sum(double x) {
    static const struct Table {
        double v[4096];
        Table() {
            v[0] = 0.0;
            for (int k = 1; k < 4096; ++k) v[k] = std::log2((double)k);
        }
    } t;
    return x < 4096.0 ? t.v[(int)x] : std::log2(x);
}

template <class NodeT>
double log2_bound(const NodeT &a) {
    const int m = a.m;
    double rs[HP_MAX_N], cs[HP_MAX_N];
    int rc[HP_MAX_N], cc[HP_MAX_N];
    for (int i = 0; i < m; ++i) rs[i] = cs[i] = 0.0, rc[i] = cc[i] = 0;
    bool zero_one = true;
    for (int i = 0; i < m; ++i)
        for (int e = a.rp[i]; e < a.rp[i + 1]; ++e) {
            rs[i] += a.v[e];
            cs[a.ci[e]] += a.v[e];
            rc[i]++;
            cc[a.ci[e]]++;
            if (a.v[e] != 1) zero_one = false;
        }
    const double *breg = bregman_table();
    double lr = 0, lc = 0, br = 0, bc = 0;
    for (int i = 0; i < m; ++i) {
        if (rs[i] == 0 || cs[i] == 0) return -INFINITY;
        lr += log2_sum(rs[i]);
        lc += log2_sum(cs[i]);
        if (zero_one) {
            br += breg[rc[i]];
            bc += breg[cc[i]];
        }
    }
    double b = std::min(lr, lc);
    if (zero_one) b = std::min(b, std::min(br, bc));
    return b + 1e-6 * (1.0 + std::fabs(b));   // rounding margin
}

// Column and row counts; returns s and the chosen line.
int min_line(const Node &a, bool *is_col, int *idx, int *colcnt) {
    const int m = a.m;
    for (int j = 0; j < m; ++j) colcnt[j] = 0;
    for (int e = 0; e < a.nnz; ++e) colcnt[a.ci[e]]++;
    int best = m + 1;
    for (int i = 0; i < m; ++i) {
        int k = a.rp[i + 1] - a.rp[i];
        if (k < best) {
            best = k;
            *is_col = false;
            *idx = i;
        }
    }
    for (int j = 0; j < m; ++j)
        if (colcnt[j] < best) {
            best = colcnt[j];
            *is_col = true;
            *idx = j;
        }
    return best;
}


// Child of row r with the pair (p, q): row r deleted; columns p, q replaced by
// ca * y_q + cb * y_p placed at min(p, q); columns above max(p, q) shift down by one.
void make_child(const Node &a, int r, int p, int q, uint64_t ca, uint64_t cb, Node *c) {
    const int m = a.m;
    const int keep = std::min(p, q), drop = std::max(p, q);
    c->m = m - 1;
    int out = 0, ri = 0;
    for (int i = 0; i < m; ++i) {
        if (i == r) continue;
        c->rp[ri++] = out;
        uint64_t aip = 0, aiq = 0;
        for (int e = a.rp[i]; e < a.rp[i + 1]; ++e) {
            if (a.ci[e] == p) aip = a.v[e];
            if (a.ci[e] == q) aiq = a.v[e];
        }
        const uint64_t mv = ca * aiq + cb * aip;
        if (mv >= HP_MAX_ENTRY) throw RangeError{"an expanded entry reached 2^22"};
        bool merged = false;
        for (int e = a.rp[i]; e < a.rp[i + 1]; ++e) {
            const int col = a.ci[e];
            if (col == p || col == q) continue;
            if (!merged && col > keep) {
                if (mv) {
                    c->ci[out] = (uint8_t)keep;
                    c->v[out++] = (uint32_t)mv;
                }
                merged = true;
            }
            c->ci[out] = (uint8_t)(col - (col > drop ? 1 : 0));
            c->v[out++] = a.v[e];
        }
        if (!merged && mv) {
            c->ci[out] = (uint8_t)keep;
            c->v[out++] = (uint32_t)mv;
        }
    }
    c->rp[ri] = out;
    c->nnz = out;
}

// Child of column cl with the row pair (p, q): column cl deleted; rows p, q replaced by
// ca * row_q + cb * row_p placed at min(p, q); rows above max(p, q) and columns above cl
// shift down by one. (Expansion (2) on the transpose, transposed back.)
void make_child_col(const Node &a, int cl, int p, int q, uint64_t ca, uint64_t cb, Node *c) {
    const int m = a.m;
    const int keep = std::min(p, q), drop = std::max(p, q);
    c->m = m - 1;
    int out = 0, ri = 0;
    for (int i = 0; i < m; ++i) {
        if (i == drop) continue;
        c->rp[ri++] = out;
        if (i != keep) {
            for (int e = a.rp[i]; e < a.rp[i + 1]; ++e) {
                const int col = a.ci[e];
                if (col == cl) continue;
                c->ci[out] = (uint8_t)(col - (col > cl ? 1 : 0));
                c->v[out++] = a.v[e];
            }
            continue;
        }
        // merged row: ca * row_q + cb * row_p, both lists sorted by column
        int eq = a.rp[q], eq_end = a.rp[q + 1], ep = a.rp[p], ep_end = a.rp[p + 1];
        while (eq < eq_end || ep < ep_end) {
            const int cq = eq < eq_end ? a.ci[eq] : 1 << 30;
            const int cp = ep < ep_end ? a.ci[ep] : 1 << 30;
            const int col = std::min(cq, cp);
            uint64_t mv = 0;
            if (cq == col) mv += ca * a.v[eq++];
            if (cp == col) mv += cb * a.v[ep++];
            if (col == cl || mv == 0) continue;
            if (mv >= HP_MAX_ENTRY) throw RangeError{"an expanded entry reached 2^22"};
            c->ci[out] = (uint8_t)(col - (col > cl ? 1 : 0));
            c->v[out++] = (uint32_t)mv;
        }
    }
    c->rp[ri] = out;
    c->nnz = out;
}

struct Pair {
    int p, q;
    uint64_t ca, cb;
};

// Pairs of expansion (2) along column cl: its nonzeros in increasing row order, an odd
// last one paired (coefficient 0) with the lowest row that is zero in this column.
int col_pairs(const Node &a, int cl, Pair *out) {
    const int m = a.m;
    int rows[HP_MAX_N];
    uint32_t vals[HP_MAX_N];
    int k = 0, zero = -1;
    for (int i = 0; i < m; ++i) {
        uint32_t v = 0;
        for (int e = a.rp[i]; e < a.rp[i + 1]; ++e)
            if (a.ci[e] == cl) {
                v = a.v[e];
                break;
            }
        if (v) {
            rows[k] = i;
            vals[k++] = v;
        } else if (zero < 0) {
            zero = i;
        }
    }
    int np = 0;
    for (int t = 0; t < k; t += 2) {
        Pair pr;
        pr.p = rows[t];
        pr.ca = vals[t];
        if (t + 1 < k) {
            pr.q = rows[t + 1];
            pr.cb = vals[t + 1];
        } else {
            pr.q = zero >= 0 ? zero : (pr.p == 0 ? 1 : 0);
            pr.cb = 0;
        }
        out[np++] = pr;
    }
    return np;
}

// Pairs of expansion (2) along row r (see the file comment).
int row_pairs(const Node &a, int r, Pair *out) {
    const int m = a.m;
    const int b = a.rp[r], e = a.rp[r + 1], k = e - b;
    int zero = -1;
    {
        int expect = 0;
        for (int t = b; t < e && zero < 0; ++t, ++expect)
            if (a.ci[t] != expect) zero = expect;
        if (zero < 0 && k < m) zero = k;
    }
    int np = 0;
    for (int t = 0; t < k; t += 2) {
        Pair pr;
        pr.p = a.ci[b + t];
        pr.ca = a.v[b + t];
        if (t + 1 < k) {
            pr.q = a.ci[b + t + 1];
            pr.cb = a.v[b + t + 1];
        } else {
            pr.q = zero >= 0 ? zero : (pr.p == 0 ? 1 : 0);
            pr.cb = 0;
        }
        out[np++] = pr;
    }
    return np;
}

// ------------------------------------------------------------------ leaf -> job packing
struct JobOut {
    std::vector<JobDesc> desc;
    std::vector<uint32_t> data;
    std::vector<double> bound;
};

// A job for the R-NW kernels. Column choice and order: the densest column is the fixed
// column of the Nijenhuis-Wilf form; the other m-1 "Gray columns" are ordered greedily so
// that each next column touches as few rows not yet touched as possible (ties: fewer
// nonzeros, then lower index). Gray column 0 flips at every other step, column j at every
// 2^(j+1)-th, so early columns should reach few rows. Row order: rows sorted by their level,
// the first Gray column touching them (rows touched by none come last). Then a flip of Gray
// column j changes only rows below hi[j] = 1 + the lowest row of column j (at most the number
// of rows of level <= j), and the kernels recompute only the suffix products of those rows.
template <class NodeT, class OutT>
static void emit_job_oriented(const NodeT &a, int problem, double root_log2, const ExpandParams &prm,
                              bool transposed, OutT *out);

// Transpose of a node (CSR of the transposed matrix, columns sorted within a row).
template <class NodeT>
static void transpose_node(const NodeT &a, NodeT *t) {
    const int m = a.m;
    t->reserve(m, a.nnz);
    t->m = m;
    t->nnz = a.nnz;
    int cnt[HP_MAX_M + 1] = {0};
    for (int e = 0; e < a.nnz; ++e) cnt[a.ci[e] + 1]++;
    for (int j = 0; j < m; ++j) cnt[j + 1] += cnt[j];
    for (int j = 0; j <= m; ++j) t->rp[j] = cnt[j];
    for (int i = 0; i < m; ++i)
        for (int e = a.rp[i]; e < a.rp[i + 1]; ++e) {
            const int pos = cnt[a.ci[e]]++;
            t->ci[pos] = (uint8_t)i;
            t->v[pos] = a.v[e];
        }
}

// Orientation of a job: per(B) = per(B^T), so a job is emitted transposed when that lets its
// first Gray column (the sparsest line other than the densest, fixed one) reach at most two
// rows while the untransposed job's cannot; the kernels' paired walk then applies.
template <class NodeT, class OutT>
void emit_job(const NodeT &a, int problem, double root_log2, const ExpandParams &prm, OutT *out) {
    const int m = a.m;
    if (m > HP_MAX_M) throw RangeError{"a job exceeds the largest supported order"};
    if (m >= 3) {
        int cc[HP_MAX_M] = {0}, rc[HP_MAX_M];
        for (int e = 0; e < a.nnz; ++e) cc[a.ci[e]]++;
        for (int i = 0; i < m; ++i) rc[i] = a.rp[i + 1] - a.rp[i];
        auto sparsest_but_densest = [m](const int *c) {
            int fixed = 0;
            for (int j = 1; j < m; ++j)
                if (c[j] > c[fixed]) fixed = j;
            int best = INT32_MAX;
            for (int j = 0; j < m; ++j)
                if (j != fixed) best = std::min(best, c[j]);
            return best;
        };
        if (sparsest_but_densest(cc) > 2 && sparsest_but_densest(rc) <= 2) {
            NodeT t;
            transpose_node(a, &t);
            emit_job_oriented(t, problem, root_log2, prm, true, out);
            return;
        }
    }
    emit_job_oriented(a, problem, root_log2, prm, false, out);
}

template <class NodeT, class OutT>
static void emit_job_oriented(const NodeT &a, int problem, double root_log2, const ExpandParams &prm,
                              bool transposed, OutT *out) {
    const int m = a.m;
    int cnt[HP_MAX_M] = {0};
    uint64_t colrows[HP_MAX_M] = {0};
    for (int i = 0; i < m; ++i)
        for (int e = a.rp[i]; e < a.rp[i + 1]; ++e) {
            cnt[a.ci[e]]++;
            colrows[a.ci[e]] |= 1ull << i;
        }
    int fixed = 0;
    for (int j = 1; j < m; ++j)
        if (cnt[j] > cnt[fixed]) fixed = j;
    double lb = std::min(log2_bound(a), root_log2);
    const double need = lb + m;   // |V| <= 2^(m-1) per, plus a sign bit
    if (lb > 180.0) throw RangeError{"the permanent bound exceeds 2^180"};
    const int auto_ring = need <= 62.5 ? HP_W64 : (need <= 126.5 ? HP_W128 : HP_RES);
    int ring = auto_ring;
    if (prm.arith == 1) ring = HP_W64;
    if (prm.arith == 2) ring = HP_W128;
    if (prm.arith == 3) ring = HP_RES;
    // a forced ring narrower than the bound allows could wrap: refuse it
    if (ring < auto_ring)
        throw RangeError{"the requested arithmetic is too narrow for this problem's bound"};
    int gray[HP_MAX_M];
    // greedy choice as a branch-free minimum of keys (new rows, nonzeros, column index). For a
    // mod 2^64 job whose first Gray column reaches at most three rows, Gray column 1 is instead
    // the sparsest column (at most three rows) that avoids those rows, if there is one: the
    // kernels then take the walk's steps four at a time.
    uint64_t avail = (m == 64 ? ~0ull : ((1ull << m) - 1)) & ~(1ull << fixed);
    uint64_t covered = 0;
    bool quad = false;
    for (int g = 0; g + 1 < m; ++g) {
        uint32_t bestkey = ~0u;
        if (g == 1 && ring == HP_W64 && m >= 5 && __builtin_popcountll(covered) <= 3) {
            for (uint64_t rest = avail; rest; rest &= rest - 1) {
                const int j = __builtin_ctzll(rest);
                const int rows = __builtin_popcountll(colrows[j]);
                if ((colrows[j] & covered) == 0 && rows >= 1 && rows <= 3)
                    bestkey = std::min(bestkey, ((uint32_t)rows << 16) | ((uint32_t)cnt[j] << 8) | (uint32_t)j);
            }
            quad = bestkey != ~0u;
        }
        if (!quad || g != 1)
            for (uint64_t rest = avail; rest; rest &= rest - 1) {
                const int j = __builtin_ctzll(rest);
                const uint32_t key = ((uint32_t)__builtin_popcountll(colrows[j] & ~covered) << 16) |
                                     ((uint32_t)cnt[j] << 8) | (uint32_t)j;
                bestkey = std::min(bestkey, key);
            }
        const int best = (int)(bestkey & 0xff);
        avail &= ~(1ull << best);
        gray[g] = best;
        covered |= colrows[best];
    }
    int slot[HP_MAX_M];
    for (int j = 0; j < m; ++j) slot[j] = -1;
    for (int g = 0; g + 1 < m; ++g) slot[gray[g]] = g;
    // row levels (the first Gray column touching the row; m-1 if none) and the row order:
    // a stable counting sort by level
    int level[HP_MAX_M];
    for (int i = 0; i < m; ++i) level[i] = m - 1;
    for (int g = m - 2; g >= 0; --g) {
        uint64_t rows = colrows[gray[g]];
        while (rows) {
            const int i = __builtin_ctzll(rows);
            rows &= rows - 1;
            level[i] = g;
        }
    }
    int order[HP_MAX_M], newrow[HP_MAX_M], lstart[HP_MAX_M + 1] = {0};
    for (int i = 0; i < m; ++i) lstart[level[i] + 1]++;
    for (int g = 0; g < m; ++g) lstart[g + 1] += lstart[g];
    for (int i = 0; i < m; ++i) order[lstart[level[i]]++] = i;
    for (int r = 0; r < m; ++r) newrow[order[r]] = r;

    uint64_t rsum[HP_MAX_M] = {0};
    int64_t bfix[HP_MAX_M] = {0};
    int nnz_gray = 0;
    for (int i = 0; i < m; ++i)
        for (int e = a.rp[i]; e < a.rp[i + 1]; ++e) {
            rsum[i] += a.v[e];
            if (a.ci[e] == fixed) bfix[i] = a.v[e];
            else ++nnz_gray;
        }
    for (int i = 0; i < m; ++i)
        if (rsum[i] >= HP_MAX_ROWSUM) throw RangeError{"a job row sum reached 2^24"};


    JobDesc d;
    const size_t base = hp_align_words(out->data.size());
    if (base / HP_DATA_ALIGN >= (1ull << 32)) throw LimitError{};
    d.data_off = (uint32_t)(base / HP_DATA_ALIGN);
    d.m = (uint8_t)m;
    d.arith = (uint8_t)ring;
    d.chunk_log2 = (uint8_t)(prm.chunk_log2 > 0 ? prm.chunk_log2 : default_chunk_log2(m));
    d.flags = 0;
    d.nnz = (uint32_t)nnz_gray;
    d.problem = (uint32_t)problem;
    if (d.chunk_log2 > m - 1) d.chunk_log2 = (uint8_t)std::max(0, m - 1);
    if (d.chunk_log2 > 12) d.chunk_log2 = 12;   // the kernels' delta tables hold 12 columns
    // at most 2^25 work items per job keep the per-job limb sums below 2^64
    if ((int)d.chunk_log2 < m - 32) d.chunk_log2 = (uint8_t)(m - 32);

    out->data.resize(base + hp_job_words(m, nnz_gray));
    uint32_t *w = out->data.data() + base;
    for (int i = 0; i < m; ++i)
        w[newrow[i]] = (uint32_t)(int32_t)(2 * bfix[i] - (int64_t)rsum[i]);
    // Gray column g holds the entries of original column gray[g]
    int gcnt[HP_MAX_M] = {0};
    for (int i = 0; i < m; ++i)
        for (int e = a.rp[i]; e < a.rp[i + 1]; ++e)
            if (a.ci[e] != fixed) gcnt[slot[a.ci[e]]]++;
    uint32_t *cs = w + m;
    uint32_t acc = 0;
    for (int g = 0; g < m - 1; ++g) {
        cs[g] = acc;
        acc += gcnt[g];
    }
    cs[m - 1] = acc;
    // hi[g]: one past the lowest job row of Gray column g, so that a flip of column g changes
    // only rows below hi[g] (at most the number of rows of level <= g)
    uint32_t *hi = w + 2 * m;
    for (int g = 0; g < m - 1; ++g) {
        int h = 0;
        uint64_t rows = colrows[gray[g]];
        while (rows) {
            const int i = __builtin_ctzll(rows);
            rows &= rows - 1;
            h = std::max(h, newrow[i] + 1);
        }
        hi[g] = (uint32_t)h;
    }
    hi[m - 1] = (uint32_t)m;
    if (m >= 2 && hi[0] <= 2) d.flags |= HP_FLAG_COL0_TWO_ROWS;
    else if (m >= 3 && hi[0] == 3) d.flags |= HP_FLAG_COL0_THREE_ROWS;
    // the four-step walks: column 0 on rows 0..a-1 (a = 2 or 3, all of level 0) and column 1
    // on rows a .. hi[1]-1 (disjoint, so all of level 1) with hi[1] <= a + 3; the kernels take
    // B as rows a..a+2 (rows that column 1 misses are common factors). Their block sums use
    // 24-bit products, exact when rows 0..a+2 have row sums below 2^7; other jobs keep the
    // paired walks.
    const uint32_t qa = hi[0];
    uint64_t qsum = 0;
    for (int i = 0; i < m; ++i)
        if (newrow[i] < (int)qa + 3) qsum = std::max(qsum, rsum[i]);
    if (quad && qsum < 128 && (qa == 2 || qa == 3) && m >= (int)qa + 3 && hi[1] > qa && hi[1] <= qa + 3 &&
        (uint32_t)__builtin_popcountll(colrows[gray[0]]) == qa &&
        (uint32_t)__builtin_popcountll(colrows[gray[1]]) == hi[1] - qa &&
        (colrows[gray[0]] & colrows[gray[1]]) == 0)
        d.flags |= HP_FLAG_QUAD;
    if (transposed) d.flags |= HP_FLAG_TRANSPOSED;
    uint32_t *ent = w + 3 * m;
    uint32_t pos[HP_MAX_M];
    for (int g = 0; g < m; ++g) pos[g] = cs[g];
    for (int r = 0; r < m; ++r) {
        const int i = order[r];
        for (int e = a.rp[i]; e < a.rp[i + 1]; ++e)
            if (a.ci[e] != fixed) {
                const int g = slot[a.ci[e]];
                ent[pos[g]++] = ((2u * a.v[e]) << 8) | (uint32_t)r;
            }
    }
    // original column of every job column (Gray slots, then the fixed one) and original row
    // of every job row (of the transposed matrix when the job is transposed): only the
    // estimator's random draws use them
    uint32_t *cm = w + 3 * m + nnz_gray;
    for (int g = 0; g < m - 1; ++g) cm[g] = (uint32_t)gray[g];
    cm[m - 1] = (uint32_t)fixed;
    uint32_t *rm = cm + m;
    for (int r = 0; r < m; ++r) rm[r] = (uint32_t)order[r];
    out->desc.push_back(d);
    out->bound.push_back(lb);
}

// ------------------------------------------------------------------ recursive expansion
struct Workspace {
    std::vector<Node> depth;   // one node buffer per depth
    std::vector<int> colcnt;
    std::atomic<size_t> *table_bytes = nullptr;   // shared by the threads of one expansion
    void init(int n, int nnz) {
        depth.assign(n + 2, Node());
        for (auto &x : depth) x.reserve(n, nnz);
        colcnt.assign(n + 1, 0);
    }
};

enum Action { DROP, LEAF, SPLIT };

Action classify(const Node &a, const ExpandParams &prm, Workspace &ws, bool *is_col, int *line) {
    if (a.m == 0) return LEAF;   // handled by the caller (per = 1)
    const int s = min_line(a, is_col, line, ws.colcnt.data());
    if (s == 0) return DROP;
    if (a.m <= prm.m_cut || a.m <= 2) return LEAF;
    if (s >= prm.s_leaf && a.m <= prm.m_cap) return LEAF;
    return SPLIT;
}

void expand_rec(int d, const ExpandParams &prm, Workspace &ws, int problem, double root_log2,
                JobOut *out) {
    const Node &a = ws.depth[d];
    bool is_col = false;
    int line = 0;
    const Action act = classify(a, prm, ws, &is_col, &line);
    if (act == DROP) return;
    if (act == LEAF) {
        const size_t w0 = out->data.size();
        emit_job(a, problem, root_log2, prm, out);
        if (prm.max_bytes && ws.table_bytes) {
            const size_t add = (out->data.size() - w0) * sizeof(uint32_t) + sizeof(JobDesc) + sizeof(double);
            if (ws.table_bytes->fetch_add(add) + add > prm.max_bytes) throw LimitError{};
        }
        return;
    }
    Pair pairs[HP_MAX_N / 2 + 1];
    const int np = is_col ? col_pairs(a, line, pairs) : row_pairs(a, line, pairs);
    for (int t = 0; t < np; ++t) {
        if (is_col)
            make_child_col(a, line, pairs[t].p, pairs[t].q, pairs[t].ca, pairs[t].cb, &ws.depth[d + 1]);
        else
            make_child(a, line, pairs[t].p, pairs[t].q, pairs[t].ca, pairs[t].cb, &ws.depth[d + 1]);
        expand_rec(d + 1, prm, ws, problem, root_log2, out);
    }
}

// Breadth-first split of the top of one tree into subtree roots (kept in tree order).
struct Pending {
    Node node;
    int problem;
    double root_log2;
};

}  // namespace

int default_chunk_log2(int m) {
    // lanes walk 2^c Gray indices (one work item = 64 lanes): one item per job up to order 19,
    // then the largest chunk the kernels' delta tables hold (the per-item set-up is then
    // spread over 4096 steps)
    int c = m - 1 - 6;
    if (c > 12) c = 12;
    if (c < 0) c = 0;
    return c;
}

std::string validate_csr(const CsrView &a) {
    if (a.n < 0 || a.n > HP_MAX_N) return "n must be in [0, 128]";
    if (a.n == 0) return "";
    if (!a.row_ptr) return "row_ptr is null";
    if (a.row_ptr[0] != 0) return "row_ptr[0] must be 0";
    for (int i = 0; i < a.n; ++i)
        if (a.row_ptr[i + 1] < a.row_ptr[i]) return "row_ptr must be non-decreasing";
    const int nnz = a.row_ptr[a.n];
    if (nnz > 0 && (!a.col_idx || !a.val)) return "col_idx/val are null";
    for (int i = 0; i < a.n; ++i)
        for (int e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) {
            if (a.col_idx[e] < 0 || a.col_idx[e] >= a.n) return "col_idx out of range";
            if (e > a.row_ptr[i] && a.col_idx[e] <= a.col_idx[e - 1])
                return "col_idx must be strictly increasing within a row";
            if (a.val[e] >= HP_MAX_ENTRY) return "entries must be below 2^22";
        }
    return "";
}

static void run_subtrees(std::vector<Pending> &pend, const ExpandParams &prm, int maxn, int maxnnz,
                         std::vector<JobOut> &outs, std::string *err, std::atomic<int> &bad) {
    std::atomic<size_t> next{0};
    std::atomic<size_t> table_bytes{0};
    int threads = prm.threads > 0 ? prm.threads : (int)std::thread::hardware_concurrency();
    threads = std::max(1, std::min(threads, 64));
    threads = (int)std::min<size_t>((size_t)threads, std::max<size_t>(pend.size(), 1));
    std::vector<std::string> errs(threads);
    auto work = [&](int tid) {
        Workspace ws;
        ws.init(maxn, maxnnz);
        ws.table_bytes = &table_bytes;
        for (;;) {
            const size_t k = next.fetch_add(1);
            if (k >= pend.size() || bad.load()) break;
            Node &root = ws.depth[0];
            const Node &src = pend[k].node;
            root.m = src.m;
            root.nnz = src.nnz;
            std::copy(src.rp.begin(), src.rp.begin() + src.m + 1, root.rp.begin());
            std::copy(src.ci.begin(), src.ci.begin() + src.nnz, root.ci.begin());
            std::copy(src.v.begin(), src.v.begin() + src.nnz, root.v.begin());
            try {
                expand_rec(0, prm, ws, pend[k].problem, pend[k].root_log2, &outs[k]);
            } catch (const RangeError &e) {
                errs[tid] = e.msg;
                bad.store(1);
            } catch (const LimitError &) {
                errs[tid] = "the job table exceeds its limit of " + std::to_string(prm.max_bytes >> 20) +
                            " MiB; raise max_table_mib or m_cut";
                bad.store(2);
            } catch (const std::bad_alloc &) {
                errs[tid] = "out of host memory during expansion";
                bad.store(2);
            }
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < threads; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &t : th) t.join();
    for (auto &e : errs)
        if (!e.empty()) *err = e;
}

int expand_problems(const std::vector<CsrView> &probs, const ExpandParams &prm, JobTable *out,
                    std::string *err) {
    const int p0 = out->n_problems;
    out->n_problems += (int)probs.size();
    out->direct_valid.resize(out->n_problems, 0);
    out->direct_value.resize(out->n_problems, 0);
    out->problem_log2_bound.resize(out->n_problems, 0.0);
    std::vector<Pending> pend;
    int maxn = 1, maxnnz = 1;
    for (size_t k = 0; k < probs.size(); ++k) {
        const CsrView &a = probs[k];
        const int pid = p0 + (int)k;
        if (a.n == 0) {
            out->direct_valid[pid] = 1;
            out->direct_value[pid] = 1;
            continue;
        }
        Node root;
        int nz = 0;
        for (int e = 0; e < a.row_ptr[a.n]; ++e) nz += a.val[e] != 0;
        root.reserve(a.n, nz);
        root.m = a.n;
        int o = 0;
        for (int i = 0; i < a.n; ++i) {
            root.rp[i] = o;
            for (int e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e)
                if (a.val[e]) {
                    root.ci[o] = (uint8_t)a.col_idx[e];
                    root.v[o++] = a.val[e];
                }
        }
        root.rp[a.n] = o;
        root.nnz = o;
        const double lb = log2_bound(root);
        out->problem_log2_bound[pid] = lb;
        if (lb == -INFINITY) {   // a zero row or column
            out->direct_valid[pid] = 1;
            out->direct_value[pid] = 0;
            continue;
        }
        if (lb > 180.0) {
            *err = "the permanent bound of a problem exceeds 2^180";
            return -2;
        }
        maxn = std::max(maxn, a.n);
        maxnnz = std::max(maxnnz, std::max(o, 1));
        pend.push_back(Pending{std::move(root), pid, lb});
    }
    // breadth-first split until there are enough subtrees for the threads
    int threads = prm.threads > 0 ? prm.threads : (int)std::thread::hardware_concurrency();
    const size_t want = (size_t)std::max(1, threads) * 16;
    Workspace ws;
    ws.init(maxn, maxnnz);
    std::vector<char> is_leaf(pend.size(), 0);
    for (int round = 0; round < 64 && pend.size() < want; ++round) {
        std::vector<Pending> nxt;
        std::vector<char> nleaf;
        bool grew = false;
        for (size_t t = 0; t < pend.size(); ++t) {
            if (is_leaf[t]) {
                nxt.push_back(std::move(pend[t]));
                nleaf.push_back(1);
                continue;
            }
            Node &a = pend[t].node;
            bool is_col = false;
            int line = 0;
            const Action act = classify(a, prm, ws, &is_col, &line);
            if (act == DROP) continue;
            if (act == LEAF) {
                nxt.push_back(std::move(pend[t]));
                nleaf.push_back(1);
                continue;
            }
            Pair pairs[HP_MAX_N / 2 + 1];
            const int np = is_col ? col_pairs(a, line, pairs) : row_pairs(a, line, pairs);
            for (int c = 0; c < np; ++c) {
                Pending ch;
                ch.node.reserve(a.m, a.nnz);
                try {
                    if (is_col)
                        make_child_col(a, line, pairs[c].p, pairs[c].q, pairs[c].ca, pairs[c].cb, &ch.node);
                    else
                        make_child(a, line, pairs[c].p, pairs[c].q, pairs[c].ca, pairs[c].cb, &ch.node);
                } catch (const RangeError &e) {
                    *err = e.msg;
                    return -2;
                }
                ch.problem = pend[t].problem;
                ch.root_log2 = pend[t].root_log2;
                nxt.push_back(std::move(ch));
                nleaf.push_back(0);
            }
            grew = true;
        }
        pend = std::move(nxt);
        is_leaf = std::move(nleaf);
        if (!grew) break;
    }
    std::vector<JobOut> outs(pend.size());
    std::atomic<int> bad{0};
    run_subtrees(pend, prm, maxn, maxnnz, outs, err, bad);
    if (bad.load()) return bad.load() == 2 ? -3 : -2;
    size_t nd = out->desc.size(), nw = hp_align_words(out->data.size());
    for (auto &o : outs) {
        nd += o.desc.size();
        nw += hp_align_words(o.data.size());
    }
    if (nw >= ((size_t)HP_DATA_ALIGN << 32)) {
        *err = "the job table exceeds 2^34 data words";
        return -3;
    }
    out->desc.reserve(nd);
    out->data.reserve(nw);
    out->log2_bound.reserve(nd);
    for (auto &o : outs) {   // append in tree order, freeing each part as it is copied
        out->data.resize(hp_align_words(out->data.size()));
        const uint32_t shift = (uint32_t)(out->data.size() / HP_DATA_ALIGN);
        for (auto d : o.desc) {
            d.data_off += shift;
            out->desc.push_back(d);
        }
        out->data.insert(out->data.end(), o.data.begin(), o.data.end());
        out->log2_bound.insert(out->log2_bound.end(), o.bound.begin(), o.bound.end());
        o = JobOut();
    }
    return 0;
}

int jobs_from_dense(int count, const int32_t *m, const int64_t *off, const uint32_t *a,
                    const ExpandParams &prm, JobTable *out, std::string *err) {
    const int p0 = out->n_problems;
    out->n_problems += count;
    out->direct_valid.resize(out->n_problems, 0);
    out->direct_value.resize(out->n_problems, 0);
    out->problem_log2_bound.resize(out->n_problems, 0.0);
    JobOut jo;
    for (int k = 0; k < count; ++k) {
        const int n = m[k];
        if (n < 1 || n > HP_MAX_M) {
            *err = "job order must be in [1, 40]";
            return -1;
        }
        Node nd;
        nd.reserve(n, n * n);
        nd.m = n;
        int o = 0;
        for (int i = 0; i < n; ++i) {
            nd.rp[i] = o;
            for (int j = 0; j < n; ++j) {
                const uint32_t v = a[off[k] + (int64_t)i * n + j];
                if (v >= HP_MAX_ENTRY) {
                    *err = "entries must be below 2^22";
                    return -1;
                }
                if (v) {
                    nd.ci[o] = (uint8_t)j;
                    nd.v[o++] = v;
                }
            }
        }
        nd.rp[n] = o;
        nd.nnz = o;
        const double lb = log2_bound(nd);
        out->problem_log2_bound[p0 + k] = lb;
        if (lb == -INFINITY) {
            out->direct_valid[p0 + k] = 1;
            out->direct_value[p0 + k] = 0;
            continue;
        }
        try {
            emit_job(nd, p0 + k, lb, prm, &jo);
        } catch (const RangeError &e) {
            *err = e.msg;
            return -2;
        } catch (const LimitError &) {
            *err = "the job table exceeds 2^34 data words";
            return -3;
        }
    }
    out->data.resize(hp_align_words(out->data.size()));
    if ((out->data.size() + jo.data.size()) / HP_DATA_ALIGN >= (1ull << 32)) {
        *err = "the job table exceeds 2^34 data words";
        return -3;
    }
    const uint32_t shift = (uint32_t)(out->data.size() / HP_DATA_ALIGN);
    for (auto d : jo.desc) {
        d.data_off += shift;
        out->desc.push_back(d);
    }
    out->data.insert(out->data.end(), jo.data.begin(), jo.data.end());
    out->log2_bound.insert(out->log2_bound.end(), jo.bound.begin(), jo.bound.end());
    return 0;
}

// ------------------------------------------------------------------ packing without the heap
namespace {

// Fixed-capacity stand-ins for the vectors of Node and JobOut, so that one dense job can be
// packed on the stack by the same code (no allocation).
template <class T, size_t N>
struct FixedVec {
    T a[N];
    size_t n = 0;
    size_t size() const { return n; }
    void resize(size_t k) {
        if (k > N) throw LimitError{};   // never for a job of order <= HP_MAX_M (sized below)
        for (size_t i = n; i < k; ++i) a[i] = T();
        n = k;
    }
    void push_back(const T &x) {
        resize(n + 1);
        a[n - 1] = x;
    }
    T *data() { return a; }
    const T *data() const { return a; }
    T &operator[](size_t i) { return a[i]; }
    const T &operator[](size_t i) const { return a[i]; }
};

struct FixedNode {
    int m = 0;
    int nnz = 0;
    int32_t rp[HP_MAX_M + 1];
    uint8_t ci[HP_MAX_M * HP_MAX_M];
    uint32_t v[HP_MAX_M * HP_MAX_M];
    void reserve(int, int) {}
};

constexpr size_t kFixedJobWords = 5 * HP_MAX_M + HP_MAX_M * HP_MAX_M + HP_DATA_ALIGN;
struct FixedJobOut {
    FixedVec<JobDesc, 1> desc;
    FixedVec<uint32_t, kFixedJobWords> data;
    FixedVec<double, 1> bound;
};

}  // namespace

size_t fixed_job_words() { return kFixedJobWords; }

int pack_dense_job(int n, const uint32_t *a, int arith, JobDesc *desc, uint32_t *data, size_t cap_words,
                   size_t *nwords, double *log2b) {
    if (n < 1 || n > HP_MAX_M || !a || !desc || !data || !nwords || !log2b) return -1;
    FixedNode nd;
    nd.m = n;
    int o = 0;
    for (int i = 0; i < n; ++i) {
        nd.rp[i] = o;
        uint64_t rs = 0;
        for (int j = 0; j < n; ++j) {
            const uint32_t v = a[(size_t)i * n + j];
            if (v >= HP_MAX_ENTRY) return -1;
            rs += v;
            if (v) {
                nd.ci[o] = (uint8_t)j;
                nd.v[o++] = v;
            }
        }
        if (rs >= HP_MAX_ROWSUM) return -2;
    }
    nd.rp[n] = o;
    nd.nnz = o;
    const double lb = log2_bound(nd);
    *log2b = lb;
    if (lb == -INFINITY) return 1;   // a zero row or column: per = 0, no job
    if (lb > 180.0) return -2;
    // the ring emit_job picks for this bound (a forced narrower ring is refused there)
    const int auto_ring = lb + n <= 62.5 ? HP_W64 : (lb + n <= 126.5 ? HP_W128 : HP_RES);
    if (arith > 0 && arith - 1 < auto_ring) return -2;
    ExpandParams prm;
    prm.arith = arith;
    FixedJobOut out;
    try {
        emit_job(nd, 0, lb, prm, &out);
    } catch (...) {
        return -2;
    }
    if (out.data.size() > cap_words || out.desc.size() != 1) return -2;
    *desc = out.desc[0];
    for (size_t k = 0; k < out.data.size(); ++k) data[k] = out.data[k];
    *nwords = out.data.size();
    return 0;
}

int pack_root_node(const CsrView &a, std::vector<uint32_t> *out, double *log2b) {
    const int n = a.n;
    Node root;
    int nz = 0;
    for (int e = 0; e < a.row_ptr[n]; ++e) nz += a.val[e] != 0;
    root.reserve(n, nz);
    root.m = n;
    int o = 0;
    for (int i = 0; i < n; ++i) {
        root.rp[i] = o;
        uint64_t rs = 0;
        for (int e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e)
            if (a.val[e]) {
                if (a.val[e] >= HP_MAX_ENTRY) return -2;
                rs += a.val[e];
                root.ci[o] = (uint8_t)a.col_idx[e];
                root.v[o++] = a.val[e];
            }
        if (rs >= HP_MAX_ROWSUM) return -2;
    }
    root.rp[n] = o;
    root.nnz = o;
    const double lb = log2_bound(root);
    *log2b = lb;
    if (lb == -INFINITY) return 1;
    out->assign(hp_node_words(n, o), 0u);
    uint32_t *w = out->data();
    float fb = (float)lb;
    if ((double)fb < lb) fb = std::nextafter(fb, INFINITY);
    uint32_t fbits;
    memcpy(&fbits, &fb, 4);
    w[0] = (uint32_t)n | ((uint32_t)o << 8);
    w[1] = fbits;
    w[2] = 0;
    w[3] = 0;
    for (int i = 0; i < n; ++i) w[4 + i / 4] |= (uint32_t)(root.rp[i + 1] - root.rp[i]) << (8 * (i & 3));
    uint32_t *ent = w + 4 + (n + 3) / 4;
    for (int e = 0; e < o; ++e) ent[e] = (root.v[e] << 8) | root.ci[e];
    return 0;
}

// Knuth's estimator of the size of the expansion tree: random root-to-leaf descents, each child
// taken with equal probability; along a path, the product of the child counts of the nodes
// above a node is an unbiased estimate of the number of nodes at that depth (here: order).
// The tree's shape depends on the nonzero pattern only (a merged entry ca q + cb p with ca, cb
// > 0 is nonzero exactly when q or p is), so the descents walk the 0-1 pattern, every child's
// entries reset to 1: no value can leave the entry range.
int estimate_tree(const CsrView &a, int T, int t, int s_leaf, int samples, uint64_t seed, double *nodes,
                  double *leaves) {
    const int n = a.n;
    for (int o = 0; o <= n; ++o) nodes[o] = leaves[o] = 0.0;
    if (n == 0 || samples <= 0) return 0;
    Node root;
    int nz = 0;
    for (int e = 0; e < a.row_ptr[n]; ++e) nz += a.val[e] != 0;
    root.reserve(n, nz);
    root.m = n;
    int o = 0;
    for (int i = 0; i < n; ++i) {
        root.rp[i] = o;
        for (int e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e)
            if (a.val[e]) {
                root.ci[o] = (uint8_t)a.col_idx[e];
                root.v[o++] = 1;
            }
    }
    root.rp[n] = o;
    root.nnz = o;
    Node cur, nxt;
    cur.reserve(n, nz);
    nxt.reserve(n, nz);
    std::vector<int> colcnt(n + 1);
    uint64_t state = seed;
    auto next_u64 = [&state]() {   // SplitMix64 (Steele, Lea and Flood)
        uint64_t z = (state += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    try {
        for (int smp = 0; smp < samples; ++smp) {
            cur.m = root.m;
            cur.nnz = root.nnz;
            std::copy(root.rp.begin(), root.rp.begin() + root.m + 1, cur.rp.begin());
            std::copy(root.ci.begin(), root.ci.begin() + root.nnz, cur.ci.begin());
            std::copy(root.v.begin(), root.v.begin() + root.nnz, cur.v.begin());
            double w = 1.0;
            for (;;) {
                bool is_col = false;
                int line = 0;
                const int s = min_line(cur, &is_col, &line, colcnt.data());
                if (s == 0) break;
                nodes[cur.m] += w;
                const bool split = cur.m > T || (cur.m > t && cur.m > 2 && s < s_leaf && s <= 4);
                if (!split) {
                    leaves[cur.m] += w;
                    break;
                }
                Pair pairs[HP_MAX_N / 2 + 1];
                const int np = is_col ? col_pairs(cur, line, pairs) : row_pairs(cur, line, pairs);
                const int k = (int)(next_u64() % (uint64_t)np);
                if (is_col)
                    make_child_col(cur, line, pairs[k].p, pairs[k].q, pairs[k].ca, pairs[k].cb, &nxt);
                else
                    make_child(cur, line, pairs[k].p, pairs[k].q, pairs[k].ca, pairs[k].cb, &nxt);
                for (int e = 0; e < nxt.nnz; ++e) nxt.v[e] = 1;
                std::swap(cur, nxt);
                w *= np;
            }
        }
    } catch (const RangeError &) {
        return -2;
    }
    for (int q = 0; q <= n; ++q) {
        nodes[q] /= samples;
        leaves[q] /= samples;
    }
    return 0;
}

}  // namespace hp
