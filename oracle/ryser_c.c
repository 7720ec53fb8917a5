/*
 * Plain Ryser permanent in C (oracle; TEST INFRASTRUCTURE ONLY: used to time a CPU
 * baseline, never by the product path).
 *
 * Ryser's formula (the method the paper cites as the first half of R-NW, Introduction):
 *   per(A) = (-1)^n * sum over column subsets S of (-1)^|S| * prod_i sum_{j in S} a_ij.
 * Subsets are enumerated in binary order and every row sum is recomputed from scratch.
 * Arithmetic is in the ring of integers modulo 2^128 (unsigned __int128). Every
 * intermediate is the exact value reduced mod 2^128, so the final residue equals per(A)
 * whenever 0 <= per(A) < 2^128 (true for non-negative matrices with per below 2^128).
 *
 * Entry point (one call evaluates a list of dense matrices on several threads):
 *   int oracle_ryser_batch(int count, const int32_t *order, const int64_t *offset,
 *                          const uint32_t *entries, uint64_t *out_lo, uint64_t *out_hi,
 *                          int threads);
 * Matrix k has order[k] (0..40) and its row-major entries start at entries[offset[k]].
 * Returns 0, or -1 on a bad argument.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdatomic.h>

typedef unsigned __int128 u128;

struct batch {
    int count;
    const int32_t *order;
    const int64_t *offset;
    const uint32_t *entries;
    uint64_t *out_lo, *out_hi;
    atomic_int next;
};

static u128 ryser(int n, const uint32_t *a)
{
    u128 total = 0;
    uint64_t nsub = (uint64_t)1 << n;
    for (uint64_t mask = 0; mask < nsub; ++mask) {
        u128 prod = 1;
        for (int i = 0; i < n; ++i) {
            u128 rowsum = 0;
            for (int j = 0; j < n; ++j)
                if ((mask >> j) & 1)
                    rowsum += a[(int64_t)i * n + j];
            prod *= rowsum;
        }
        if (__builtin_popcountll(mask) & 1)
            total -= prod;
        else
            total += prod;
    }
    if (n & 1)
        total = (u128)0 - total;
    return total;
}

static void *worker(void *arg)
{
    struct batch *b = (struct batch *)arg;
    for (;;) {
        int k = atomic_fetch_add(&b->next, 1);
        if (k >= b->count)
            break;
        u128 v = ryser(b->order[k], b->entries + b->offset[k]);
        b->out_lo[k] = (uint64_t)v;
        b->out_hi[k] = (uint64_t)(v >> 64);
    }
    return 0;
}

int oracle_ryser_batch(int count, const int32_t *order, const int64_t *offset,
                       const uint32_t *entries, uint64_t *out_lo, uint64_t *out_hi, int threads)
{
    if (count < 0 || threads < 1 || threads > 1024)
        return -1;
    for (int k = 0; k < count; ++k)
        if (order[k] < 0 || order[k] > 40)
            return -1;
    struct batch b = {count, order, offset, entries, out_lo, out_hi, 0};
    pthread_t tid[1024];
    int started = 0;
    for (int t = 0; t < threads; ++t)
        if (pthread_create(&tid[t], 0, worker, &b) == 0)
            ++started;
    if (started == 0)
        worker(&b);
    for (int t = 0; t < started; ++t)
        pthread_join(tid[t], 0);
    return 0;
}
