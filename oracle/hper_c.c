/*
 * Algorithm H_per in C (oracle; TEST INFRASTRUCTURE ONLY: never used by the product path).
 *
 * Section 2.1 of the paper: with s the minimal number of nonzeros in a row or column,
 * if n > 2 and s < 5 the matrix is split by expansion (2) and the permanents of the
 * children are added; otherwise the permanent is evaluated directly (R-NW in the
 * paper; here plain Ryser, binary subset order, row sums recomputed per subset).
 *
 * Expansion (2) along a row whose nonzeros, in column order, are v1, v2, ... at columns
 * p1, p2, ...: the pair (p1, p2) gives the child with the row deleted and columns p1, p2
 * replaced by the single column v1*y(p2) + v2*y(p1); (p3, p4) gives the next child, and so
 * on (repeating the expansion on the remainder matrix A3 while the row has nonzeros left).
 * An odd last nonzero is paired, with coefficient 0, with the lowest-index column that is
 * zero in this row (or the lowest other column if there is none). A column is expanded by the same rule on the transpose. Ties for the
 * minimal line go to rows first, then to the lowest index; n = 0 gives 1, n = 1 gives a11,
 * n = 2 gives a11*a22 + a12*a21.
 *
 * Arithmetic: entries are uint64 (checked to stay below 2^62), permanents are computed in
 * the ring of integers mod 2^128; the result is exact whenever 0 <= per(A) < 2^128.
 *
 *   int oracle_hper_batch(int count, const int32_t *order, const int64_t *offset,
 *                         const uint64_t *entries, uint64_t *out_lo, uint64_t *out_hi,
 *                         int threads);
 * Matrix k has order[k] (0..128), row-major entries from entries[offset[k]]. The top of
 * each expansion tree is split breadth-first into independent subtrees that the threads
 * share. Returns 0; -1 on a bad argument; -2 if an entry grew past 2^62.
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef uint64_t ent;

static atomic_int g_overflow;

static u128 ryser_dense(int n, const ent *a)
{
    u128 total = 0;
    uint64_t nsub = (uint64_t)1 << n;
    for (uint64_t mask = 0; mask < nsub; ++mask) {
        u128 prod = 1;
        for (int i = 0; i < n; ++i) {
            u128 rowsum = 0;
            for (int j = 0; j < n; ++j)
                if ((mask >> j) & 1)
                    rowsum += a[i * n + j];
            prod *= rowsum;
        }
        if (__builtin_popcountll(mask) & 1)
            total -= prod;
        else
            total += prod;
    }
    return (n & 1) ? (u128)0 - total : total;
}

/* The line with the fewest nonzeros: *is_col, *idx; returns s. */
static int min_line(int n, const ent *a, int *is_col, int *idx)
{
    int best = n + 1;
    for (int i = 0; i < n; ++i) {
        int k = 0;
        for (int j = 0; j < n; ++j)
            k += a[i * n + j] != 0;
        if (k < best) {
            best = k;
            *is_col = 0;
            *idx = i;
        }
    }
    for (int j = 0; j < n; ++j) {
        int k = 0;
        for (int i = 0; i < n; ++i)
            k += a[i * n + j] != 0;
        if (k < best) {
            best = k;
            *is_col = 1;
            *idx = j;
        }
    }
    return best;
}

/* Write the child of the pair (p, q) of row r into c ((n-1)x(n-1)); a is n x n, row-major.
 * With is_col the roles of rows and columns are exchanged (expansion of the transpose). */
static void make_child(int n, const ent *a, int is_col, int r, int p, int q, int odd, ent *c)
{
#define AT(i, j) (is_col ? a[(j) * n + (i)] : a[(i) * n + (j)])
    ent ca = AT(r, p), cb = odd ? 0 : AT(r, q);
    int keep = p < q ? p : q, drop = p < q ? q : p;
    int m = n - 1;
    int ci = 0;
    for (int i = 0; i < n; ++i) {
        if (i == r)
            continue;
        int cj = 0;
        for (int j = 0; j < n; ++j) {
            if (j == drop)
                continue;
            ent v;
            if (j == keep) {
                u128 w = (u128)ca * AT(i, q) + (u128)cb * AT(i, p);
                if (w >> 62)
                    atomic_store(&g_overflow, 1);
                v = (ent)w;
            } else {
                v = AT(i, j);
            }
            if (is_col)
                c[cj * m + ci] = v;
            else
                c[ci * m + cj] = v;
            ++cj;
        }
        ++ci;
    }
#undef AT
}

/* Pairs of the expansion along line (is_col, r): fills p[], q[] and odd (1 when the last
 * pair is an odd nonzero with a coefficient-0 partner); returns the child count. */
static int pairs_of(int n, const ent *a, int is_col, int r, int *p, int *q, int *odd)
{
    int nz[128], k = 0, zero = -1;
    for (int j = 0; j < n; ++j) {
        ent v = is_col ? a[j * n + r] : a[r * n + j];
        if (v)
            nz[k++] = j;
        else if (zero < 0)
            zero = j;
    }
    int c = 0;
    *odd = 0;
    for (int t = 0; t < k; t += 2) {
        p[c] = nz[t];
        if (t + 1 < k) {
            q[c] = nz[t + 1];
        } else {
            q[c] = zero >= 0 ? zero : (nz[t] == 0 ? 1 : 0);
            *odd = 1;
        }
        ++c;
    }
    return c;
}

static u128 hper(int n, const ent *a)
{
    if (n == 0)
        return 1;
    if (n == 1)
        return a[0];
    if (n == 2)
        return (u128)a[0] * a[3] + (u128)a[1] * a[2];
    int is_col = 0, r = 0;
    int s = min_line(n, a, &is_col, &r);
    if (s == 0)
        return 0;
    if (s >= 5)
        return ryser_dense(n, a);
    int p[3], q[3], odd;
    int nc = pairs_of(n, a, is_col, r, p, q, &odd);
    ent *child = (ent *)malloc(sizeof(ent) * (n - 1) * (n - 1));
    u128 sum = 0;
    for (int t = 0; t < nc; ++t) {
        make_child(n, a, is_col, r, p[t], q[t], odd && t == nc - 1, child);
        sum += hper(n - 1, child);
    }
    free(child);
    return sum;
}

/* ---------------------------------------------------------------- parallel driver */
struct task {
    int n;
    ent *a;
    int owner;          /* index of the input matrix */
};

struct pool {
    struct task *tasks;
    int ntask;
    atomic_int next;
    u128 *partial;      /* per task */
};

static void *worker(void *arg)
{
    struct pool *pl = (struct pool *)arg;
    for (;;) {
        int k = atomic_fetch_add(&pl->next, 1);
        if (k >= pl->ntask)
            break;
        pl->partial[k] = hper(pl->tasks[k].n, pl->tasks[k].a);
    }
    return 0;
}

static int push(struct task **v, int *len, int *cap, struct task t)
{
    if (*len == *cap) {
        *cap = *cap ? 2 * *cap : 256;
        *v = (struct task *)realloc(*v, sizeof(struct task) * *cap);
    }
    (*v)[(*len)++] = t;
    return 0;
}

int oracle_hper_batch(int count, const int32_t *order, const int64_t *offset,
                      const uint64_t *entries, uint64_t *out_lo, uint64_t *out_hi, int threads)
{
    if (count < 0 || threads < 1 || threads > 1024)
        return -1;
    for (int k = 0; k < count; ++k)
        if (order[k] < 0 || order[k] > 128)
            return -1;
    atomic_store(&g_overflow, 0);
    u128 *direct = (u128 *)calloc(count ? count : 1, sizeof(u128));
    /* Split the top of every tree breadth-first until there are enough subtrees. */
    struct task *cur = 0, *nxt = 0;
    int ncur = 0, ccur = 0;
    for (int k = 0; k < count; ++k) {
        int n = order[k];
        ent *a = (ent *)malloc(sizeof(ent) * (n ? n * n : 1));
        memcpy(a, entries + offset[k], sizeof(ent) * n * n);
        struct task t = {n, a, k};
        push(&cur, &ncur, &ccur, t);
    }
    int want = 64 * threads;
    for (int round = 0; round < 40 && ncur < want; ++round) {
        int nn = 0, cn = 0;
        nxt = 0;
        for (int t = 0; t < ncur; ++t) {
            int n = cur[t].n;
            ent *a = cur[t].a;
            int is_col = 0, r = 0;
            int s = n > 2 ? min_line(n, a, &is_col, &r) : 5;
            if (n <= 2 || s == 0 || s >= 5) {
                push(&nxt, &nn, &cn, cur[t]);   /* evaluated as a whole later */
                continue;
            }
            int p[3], q[3], odd;
            int nc = pairs_of(n, a, is_col, r, p, q, &odd);
            for (int c = 0; c < nc; ++c) {
                ent *ch = (ent *)malloc(sizeof(ent) * (n - 1) * (n - 1));
                make_child(n, a, is_col, r, p[c], q[c], odd && c == nc - 1, ch);
                struct task tc = {n - 1, ch, cur[t].owner};
                push(&nxt, &nn, &cn, tc);
            }
            free(a);
        }
        free(cur);
        cur = nxt;
        ncur = nn;
        ccur = cn;
    }
    struct pool pl = {cur, ncur, 0, (u128 *)calloc(ncur ? ncur : 1, sizeof(u128))};
    pthread_t tid[1024];
    int started = 0;
    for (int t = 0; t < threads; ++t)
        if (pthread_create(&tid[t], 0, worker, &pl) == 0)
            ++started;
    if (started == 0)
        worker(&pl);
    for (int t = 0; t < started; ++t)
        pthread_join(tid[t], 0);
    for (int t = 0; t < ncur; ++t) {
        direct[cur[t].owner] += pl.partial[t];
        free(cur[t].a);
    }
    for (int k = 0; k < count; ++k) {
        out_lo[k] = (uint64_t)direct[k];
        out_hi[k] = (uint64_t)(direct[k] >> 64);
    }
    free(cur);
    free(pl.partial);
    free(direct);
    return atomic_load(&g_overflow) ? -2 : 0;
}
