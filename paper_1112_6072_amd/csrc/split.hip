// Device continuation of Algorithm H_per (Section 2.1) below the host's (or the device
// expansion's) cut-off, R-NW on the leaves it reaches, and their exact sum per job (Step 4 of
// Algorithm PH, inside one job).
//
// One wave takes one job (a sub-matrix B of order m <= HP_SPLIT_MAX_M) from a queue and
// rebuilds it densely in its LDS region, from the R-NW job table of the host expansion or from
// a node of the device expansion (hp_node_words). It walks the H_per expansion tree of B depth
// first. At a node of order o, s is the smallest number of nonzeros in a row or a column
// (ties: rows first, then the lowest index). s = 0 drops the node (per = 0); a node with
// o <= t (the target order), o <= 2 or s >= s_leaf is a leaf; otherwise expansion (2) along
// that line gives ceil(s/2) <= 2 children of order o - 1: consecutive nonzeros of the line are
// paired and each pair's two columns (rows, for a column line) merged with crossed weights,
// an odd last nonzero paired at weight 0 with the lowest zero of the line. This is the rule of
// the host expansion. The nodes on the current path all have different orders, so each order
// has one LDS slot: the node of order o and its control state (line, pairs, next child) live
// at slot o, with the nonzero bit masks of its rows and columns and its row sums, which the
// child construction keeps up to date (so the line choice and the bound checks cost O(1) per
// lane). A split whose children would hold an entry >= 2^22 or a row sum >= 2^24 is not made:
// the node becomes a leaf (the bounds the host keeps for every job).
//
// Exactness. Each leaf is normalised on its own: a leaf of order p is evaluated with the
// doubled Nijenhuis-Wilf form of Ryser's formula (fixed column p - 1, Gray columns 0..p-2),
//     V = sum_k (-1)^k prod_i f_i(gray(k)) = (-1)^(p-1) 2^(p-1) per(leaf),
// modulo 2^64, which is exact when per(leaf) 2^(p-1) < 2^63. A proven bound decides it: the
// smaller of the job's bound (per(leaf) <= per(B), all entries being non-negative) and the
// leaf's product of row sums. Then per(leaf) = (-1)^(p-1) V / 2^(p-1), checked (non-negative,
// divisible; a failure is counted and reported, never summed), and added to the job's sum in
// 128-bit integers. For a leaf the bound does not admit, and for leaves above order 16, the
// wave records the job, the leaf's order and the path of child choices to it, and a second
// kernel replays the path and evaluates the leaf modulo 2^128 (exact for jobs whose bound is
// below 2^102, which the host requires).
//
// Lane z of a leaf of order p >= 7 walks the 2^(p-7) Gray indices of chunk z, odd chunks
// backwards. Then at step s every lane flips Gray column ctz(s) and adds it exactly when bit
// ctz(s) + 1 of s is clear (both hold in either direction of the reflected code), no lane's
// start subset holds a column below p - 7, and the term of step s has the sign (-1)^(s + z).
// Rows beyond p are padded with f = 1. Leaves have order p >= t >= 7.
//
// Modular mode (SplitArgs.modps, a prime p < 2^18 per problem; nodes of the device expansion in
// the same mode): merged entries are reduced modulo the job's problem's p, every leaf is evaluated modulo p in FP64 (exact:
// operands and products stay below 2^53) and normalised with the inverse of 2^(p-1), and the
// sums are residues: per(B) mod p.
//
// Results: per-job values (JobAcc, flagged normalised) for the host's job tables; for the
// device expansion's nodes, each wave sums its jobs' values per problem and adds them into the
// problem accumulators (ProbAcc), and per-node values are written only when asked for.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hperm_internal.h"
#include "kernels.h"

namespace hp {
namespace {

constexpr int SW = 64;                   // one wave per block
constexpr int SMAX = HP_SPLIT_MAX_M;     // largest job order
constexpr int CTL = 8;                   // control words of an undo record
constexpr int PMAX = 16;                 // widest leaf the main kernel evaluates
// Words per Gray column of a leaf's delta table (every row; a multiple of 4 for the 16-byte
// loads), for jobs of order <= mm.
__host__ __device__ constexpr int dstride(int mm) { return mm <= 20 ? 20 : 24; }
static_assert(dstride(SMAX) >= SMAX && dstride(SMAX) % 4 == 0, "a delta-table column holds every row");

__host__ __device__ constexpr int align4(int w) { return (w + 3) & ~3; }

typedef unsigned __int128 u128;

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    return (uint64_t)uni((uint32_t)x) | ((uint64_t)uni((uint32_t)(x >> 32)) << 32);
}

// LDS writes of some lanes made visible to the other lanes of the wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
    for (int o = 32; o; o >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, o);
    return v;
}

__device__ __forceinline__ float wave_sumf(float v) {
    for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Inclusive prefix sum over the lanes.
__device__ __forceinline__ uint32_t wave_scan(uint32_t v, int lane) {
    for (int o = 1; o < SW; o <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)v, o);
        if (lane >= o) v += u;
    }
    return v;
}

// 128-bit sum over the lanes (as four 32-bit limb sums).
__device__ __forceinline__ u128 wave_sum128(u128 v) {
    const uint64_t a = wave_sum64((uint32_t)v), b = wave_sum64((uint32_t)(v >> 32));
    const uint64_t c = wave_sum64((uint32_t)(v >> 64)), d = wave_sum64((uint32_t)(v >> 96));
    return (u128)a + ((u128)b << 32) + ((u128)c << 64) + ((u128)d << 96);
}

// Among the lanes with `valid`, the lowest one holding the smallest count (count < 32): a
// search over the count's bits with ballots (no LDS round trips). Writes that count.
__device__ __forceinline__ uint32_t argmin_lane(uint32_t count, bool valid, uint32_t *minval) {
    uint64_t set = __ballot(valid);
#pragma unroll
    for (int b = 4; b >= 0; --b) {
        const uint64_t zero = __ballot(((count >> b) & 1u) == 0) & set;
        if (zero) set = zero;
    }
    const uint32_t w = (uint32_t)__builtin_ctzll(set);
    *minval = (uint32_t)__builtin_amdgcn_readlane((int)count, (int)w);
    return w;
}

// The product of two row values, exact in 64 bits (|x|, |y| < 2^24), kept as one value: the
// empty asm stops the compiler from re-associating a product of such pairs into a chain of
// 64 x 32-bit multiplies (five instructions each instead of one here).
__device__ __forceinline__ uint64_t pmul(int32_t x, int32_t y) {
    int64_t p = (int64_t)x * (int64_t)y;
    asm("" : "+v"(p));
    return (uint64_t)p;
}

// Product modulo 2^64 of rows LO..R-1 (R - LO even, at least 2): the pair products, then a
// balanced tree of 64-bit multiplies.
template <int R, int LO>
__device__ __forceinline__ uint64_t pair_product(const int32_t (&f)[R]) {
    constexpr int N = (R - LO) / 2;
    uint64_t q[N];
#pragma unroll
    for (int k = 0; k < N; ++k) q[k] = pmul(f[LO + 2 * k], f[LO + 2 * k + 1]);
#pragma unroll
    for (int w = 1; w < N; w *= 2) {
#pragma unroll
        for (int k = 0; k + w < N; k += 2 * w) q[k] *= q[k + w];
    }
    return q[0];
}

// The same product modulo 2^128 (replay kernel).
template <int R>
__device__ __forceinline__ u128 row_product128(const int32_t (&f)[R]) {
    u128 p = (u128)(__int128)((int64_t)f[0] * (int64_t)f[1]);
#pragma unroll
    for (int k = 1; k < R / 2; ++k) p *= (u128)(__int128)((int64_t)f[2 * k] * (int64_t)f[2 * k + 1]);
    return p;
}

// Leaf tables of the main kernel (one per wave): Gray column j's deltas 2 b_ij at D + j PM,
// their negatives at D + TNEG + j PM, the base values at D + 2 TNEG; rows p..PM-1 padded (delta
// 0, base 1).
constexpr int PM = PMAX;                 // table stride: rows of the widest leaf
static_assert(SW == 4 * PM, "leaf tables: one row per lane in each quarter of the wave");
constexpr int TNEG = (PMAX - 1) * PMAX;
__host__ __device__ constexpr int leaf_table_words() { return 2 * TNEG + PMAX; }

// f += the deltas at d (a + or - table column), R rows.
template <int R>
__device__ __forceinline__ void add_rows(int32_t (&f)[R], const int32_t *d) {
#pragma unroll
    for (int i = 0; i < R; i += 4) {
        const int4 w = *(const int4 *)(d + i);
        f[i] += w.x;
        f[i + 1] += w.y;
        f[i + 2] += w.z;
        f[i + 3] += w.w;
    }
}

// Row values of this lane's first Gray index (no Gray column below p - 7 is set in it).
template <int R>
__device__ __forceinline__ void start_rows(int32_t (&f)[R], int p, int lane, const int32_t *D) {
    const int c = p - 7;
    const uint32_t L = 1u << c;
    const uint32_t kfirst = (lane & 1) ? (uint32_t)lane * L + L - 1 : (uint32_t)lane * L;
    const uint32_t s0 = kfirst ^ (kfirst >> 1);
    const int32_t *base = D + 2 * TNEG;
#pragma unroll
    for (int i = 0; i < R; i += 4) {
        const int4 w = *(const int4 *)(base + i);
        f[i] = w.x;
        f[i + 1] = w.y;
        f[i + 2] = w.z;
        f[i + 3] = w.w;
    }
#pragma unroll 1
    for (int j = c; j < p - 1; ++j) {
        const int32_t in = -(int32_t)((s0 >> j) & 1);   // all ones when Gray column j is in
        const int32_t *dj = D + j * PM;
#pragma unroll
        for (int i = 0; i < R; i += 4) {
            const int4 w = *(const int4 *)(dj + i);
            f[i] += w.x & in;
            f[i + 1] += w.y & in;
            f[i + 2] += w.z & in;
            f[i + 3] += w.w & in;
        }
    }
}

// The table column of the flip at step s >= 1 (Gray column ctz(s), added when bit ctz(s) + 1
// of s is clear).
__device__ __forceinline__ const int32_t *flip_column(const int32_t *D, uint32_t s) {
    const int j = __builtin_ctz(s);
    return D + j * PM + (((s >> (j + 1)) & 1) ? TNEG : 0);
}

// This lane's share of V for a leaf of order p (7 <= p <= R): one term per step.
template <int R>
__device__ __forceinline__ uint64_t walk_plain(int p, int lane, const int32_t *D) {
    const uint32_t L = 1u << (p - 7);
    int32_t f[R];
    start_rows<R>(f, p, lane, D);
    uint64_t acc0 = pair_product<R, 0>(f), acc1 = 0;
    for (uint32_t s = 1; s < L; s += 2) {
        add_rows<R>(f, flip_column(D, s));   // odd steps flip Gray column 0
        acc1 += pair_product<R, 0>(f);
        if (s + 1 < L) {
            add_rows<R>(f, flip_column(D, s + 1));
            acc0 += pair_product<R, 0>(f);
        }
    }
    return (lane & 1) ? acc1 - acc0 : acc0 - acc1;
}

// The same share with the steps taken in pairs (8 <= p <= R; Gray column 0 touches only rows
// 0..BB-1). Steps s (even) and s + 1 differ only by Gray column 0, so their terms are A*P and
// B*P with P the product of rows BB..R-1 and A, B the products of rows 0..BB-1 before and after
// the flip: each pair costs one product of the other rows and one of the small block twice.
template <int R, int BB>
__device__ __forceinline__ uint64_t walk_paired(int p, int lane, const int32_t *D) {
    const uint32_t L = 1u << (p - 7);
    int32_t f[R];
    start_rows<R>(f, p, lane, D);
    int32_t dp[BB], dn[BB];   // Gray column 0's deltas and their negatives
#pragma unroll
    for (int i = 0; i < BB; ++i) {
        dp[i] = D[i];
        dn[i] = D[TNEG + i];
    }
    uint64_t acc = 0;
    for (uint32_t s = 0;;) {
        const bool add0 = (((s + 1) >> 1) & 1) == 0;   // step s + 1 adds Gray column 0
        int32_t g[BB];
#pragma unroll
        for (int i = 0; i < BB; ++i) g[i] = f[i] + (add0 ? dp[i] : dn[i]);
        const uint64_t rest = pair_product<R, BB>(f);
        uint64_t a, b;
        if constexpr (BB == 2) {
            a = pmul(f[0], f[1]);
            b = pmul(g[0], g[1]);
        } else {
            a = pmul(f[0], f[1]) * pmul(f[2], f[3]);
            b = pmul(g[0], g[1]) * pmul(g[2], g[3]);
        }
        acc += (a - b) * rest;
#pragma unroll
        for (int i = 0; i < BB; ++i) f[i] = g[i];   // step s + 1 leaves Gray column 0 flipped
        s += 2;
        if (s >= L) break;
        add_rows<R>(f, flip_column(D, s));          // step s flips Gray column ctz(s) >= 1
    }
    return (lane & 1) ? (uint64_t)0 - acc : acc;
}

// Product modulo 2^64 of rows LO..R-1 (any count >= 2).
template <int R, int LO>
__device__ __forceinline__ uint64_t rest_product(const int32_t (&f)[R]) {
    if constexpr ((R - LO) % 2 == 0) return pair_product<R, LO>(f);
    else return pair_product<R, LO + 1>(f) * (uint64_t)(int64_t)f[LO];
}

// Product modulo 2^64 of N = 2 or 3 row values.
template <int N>
__device__ __forceinline__ uint64_t small_product(const int32_t (&x)[N]) {
    if constexpr (N == 2) return pmul(x[0], x[1]);
    else return pmul(x[0], x[1]) * (uint64_t)(int64_t)x[2];
}

// The same share with the steps taken in blocks of four (9 <= p <= R): Gray column 0 touches
// only rows 0..NA-1 and Gray column 1 only rows NA..NA+NB-1 (disjoint; filler rows that
// neither touches pad the two groups). In the block of steps 4q .. 4q+3 every other column is
// fixed and the four terms take both values of columns 0 and 1, with signs (-1)^(q+z) times
// +, -, +, - in the reflected code's order, so their sum factors as
//     (-1)^(q+z) (A0 - A1) (B0 - B1) P,
// where A0, A1 are the products of rows 0..NA-1 without and with column 0, B0, B1 those of
// rows NA..NA+NB-1 without and with column 1, P the product of the other rows, all taken with
// columns 0 and 1 out (the values h). A block costs one product of the other rows, four small
// ones and two multiplies, where the paired walk takes two products of the other rows.
template <int R, int NA, int NB>
__device__ __forceinline__ uint64_t walk_quad(int p, int lane, const int32_t *D) {
    const uint32_t L = 1u << (p - 7);   // a multiple of 4
    int32_t h[R];
    start_rows<R>(h, p, lane, D);       // no Gray column below p - 7 is set: h itself
    int32_t da[NA], db[NB];             // column 0's deltas on rows 0..NA-1, column 1's on NA..
#pragma unroll
    for (int i = 0; i < NA; ++i) da[i] = D[i];
#pragma unroll
    for (int i = 0; i < NB; ++i) db[i] = D[PM + NA + i];
    uint64_t acc = 0;
    for (uint32_t s = 0;;) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            int32_t a0[NA], a1[NA], b0[NB], b1[NB];
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                a0[i] = h[i];
                a1[i] = h[i] + da[i];
            }
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                b0[i] = h[NA + i];
                b1[i] = h[NA + i] + db[i];
            }
            const uint64_t x = (small_product<NA>(a0) - small_product<NA>(a1)) *
                               (small_product<NB>(b0) - small_product<NB>(b1)) * rest_product<R, NA + NB>(h);
            acc = half ? acc - x : acc + x;   // blocks alternate in sign
            s += 4;
            if (s >= L) return (lane & 1) ? (uint64_t)0 - acc : acc;
            add_rows<R>(h, flip_column(D, s));   // step s flips Gray column ctz(s) >= 2
        }
    }
}

// The replay kernel's walk modulo 2^128 over a table of stride ds (deltas only; a subtraction
// is a branch: the replay is rare).
template <int R>
__device__ __forceinline__ void add_rows_dir(int32_t (&f)[R], const int32_t *d, bool add) {
    int32_t v[R];
#pragma unroll
    for (int i = 0; i < R; i += 4) {
        const int4 w = *(const int4 *)(d + i);
        v[i] = w.x;
        v[i + 1] = w.y;
        v[i + 2] = w.z;
        v[i + 3] = w.w;
    }
    if (add) {
#pragma unroll
        for (int i = 0; i < R; ++i) f[i] += v[i];
    } else {
#pragma unroll
        for (int i = 0; i < R; ++i) f[i] -= v[i];
    }
}

template <int R>
__device__ __forceinline__ u128 walk_plain128(int p, int lane, const int32_t *D, const int32_t *base, int ds) {
    const uint32_t L = 1u << (p - 7);
    int32_t f[R];
    {
        const int c = p - 7;
        const uint32_t kfirst = (lane & 1) ? (uint32_t)lane * L + L - 1 : (uint32_t)lane * L;
        const uint32_t s0 = kfirst ^ (kfirst >> 1);
#pragma unroll
        for (int i = 0; i < R; ++i) f[i] = base[i];
        for (int j = c; j < p - 1; ++j) {
            const int32_t in = -(int32_t)((s0 >> j) & 1);
#pragma unroll
            for (int i = 0; i < R; ++i) f[i] += D[j * ds + i] & in;
        }
    }
    u128 acc0 = row_product128<R>(f), acc1 = 0;
    for (uint32_t s = 1; s < L; s += 2) {
        add_rows_dir<R>(f, D, ((s >> 1) & 1) == 0);
        acc1 += row_product128<R>(f);
        if (s + 1 < L) {
            const uint32_t s2 = s + 1;
            const int j = __builtin_ctz(s2);
            add_rows_dir<R>(f, D + j * ds, ((s2 >> (j + 1)) & 1) == 0);
            acc0 += row_product128<R>(f);
        }
    }
    return (lane & 1) ? acc1 - acc0 : acc0 - acc1;
}

// ---- modular mode: per(B) modulo a prime p < 2^18 (the permanental polynomial's residues) ----
// FP64 arithmetic: every operand and product below 2^53 is exact, and x mod p is
// x - floor(x / p) p with the quotient from the rounded reciprocal off by at most one, which
// two corrections absorb.
struct ModP {
    double p, pinv;
};
__device__ __forceinline__ double red_f(double x, const ModP &m) {   // |x| < 2^53 -> [0, p)
    double r = __builtin_fma(-floor(x * m.pinv), m.p, x);
    r = r < 0.0 ? r + m.p : r;
    return r >= m.p ? r - m.p : r;
}

// The product of the R row values modulo p: exact pair products (|f| < 2^24), reduced, chained.
template <int R>
__device__ __forceinline__ double mod_product(const int32_t (&f)[R], const ModP &m) {
    double r = red_f((double)f[0] * (double)f[1], m);
#pragma unroll
    for (int k = 1; k < R / 2; ++k) r = red_f(r * red_f((double)f[2 * k] * (double)f[2 * k + 1], m), m);
    return r;
}

// This lane's share of V modulo p (in [0, p)) for a leaf of order 7 <= p <= R in the main
// kernel's tables (one term per step).
template <int R>
__device__ __forceinline__ uint64_t walk_mod(int p, int lane, const int32_t *D, const ModP &m) {
    const uint32_t L = 1u << (p - 7);
    int32_t f[R];
    start_rows<R>(f, p, lane, D);
    double acc0 = mod_product<R>(f, m), acc1 = 0.0;
    for (uint32_t s = 1; s < L; s += 2) {
        add_rows<R>(f, flip_column(D, s));
        acc1 += mod_product<R>(f, m);
        acc1 = acc1 >= m.p ? acc1 - m.p : acc1;
        if (s + 1 < L) {
            add_rows<R>(f, flip_column(D, s + 1));
            acc0 += mod_product<R>(f, m);
            acc0 = acc0 >= m.p ? acc0 - m.p : acc0;
        }
    }
    double v = (lane & 1) ? acc1 - acc0 : acc0 - acc1;
    v = v < 0.0 ? v + m.p : v;
    return (uint64_t)v;
}

// The same over the replay kernel's tables (stride ds, base separate).
template <int R>
__device__ __forceinline__ uint64_t walk_mod_wide(int p, int lane, const int32_t *D, const int32_t *base, int ds,
                                                  const ModP &m) {
    const uint32_t L = 1u << (p - 7);
    int32_t f[R];
    {
        const int c = p - 7;
        const uint32_t kfirst = (lane & 1) ? (uint32_t)lane * L + L - 1 : (uint32_t)lane * L;
        const uint32_t s0 = kfirst ^ (kfirst >> 1);
#pragma unroll
        for (int i = 0; i < R; ++i) f[i] = base[i];
        for (int j = c; j < p - 1; ++j) {
            const int32_t in = -(int32_t)((s0 >> j) & 1);
#pragma unroll
            for (int i = 0; i < R; ++i) f[i] += D[j * ds + i] & in;
        }
    }
    double acc0 = mod_product<R>(f, m), acc1 = 0.0;
    for (uint32_t s = 1; s < L; s += 2) {
        add_rows_dir<R>(f, D, ((s >> 1) & 1) == 0);
        acc1 += mod_product<R>(f, m);
        acc1 = acc1 >= m.p ? acc1 - m.p : acc1;
        if (s + 1 < L) {
            const uint32_t s2 = s + 1;
            const int j = __builtin_ctz(s2);
            add_rows_dir<R>(f, D + j * ds, ((s2 >> (j + 1)) & 1) == 0);
            acc0 += mod_product<R>(f, m);
            acc0 = acc0 >= m.p ? acc0 - m.p : acc0;
        }
    }
    double v = (lane & 1) ? acc1 - acc0 : acc0 - acc1;
    v = v < 0.0 ? v + m.p : v;
    return (uint64_t)v;
}

// The product of rows LO..R-1 modulo p (at least two rows; |f| < 2^23): exact pair products
// reduced, chained (an odd count takes its first row as a single factor).
template <int R, int LO>
__device__ __forceinline__ double mod_rows(const int32_t (&f)[R], const ModP &m) {
    constexpr int K = R - LO;
    constexpr int P0 = LO + (K & 1);   // first row of the pairs
    double r = red_f((double)f[P0] * (double)f[P0 + 1], m);
#pragma unroll
    for (int k = P0 + 2; k < R; k += 2) r = red_f(r * red_f((double)f[k] * (double)f[k + 1], m), m);
    if constexpr (K & 1) r = red_f(r * (double)f[LO], m);
    return r;
}

// The product of N = 2 or 3 row values modulo p.
template <int N>
__device__ __forceinline__ double mod_small(const int32_t (&x)[N], const ModP &m) {
    double r = red_f((double)x[0] * (double)x[1], m);
    if constexpr (N == 3) r = red_f(r * (double)x[2], m);
    return r;
}

// The four-step walk (walk_quad) modulo p: the block sum (-1)^(q+z) (A0 - A1)(B0 - B1) P with
// every factor reduced. Returns this lane's share in [0, p).
template <int R, int NA, int NB>
__device__ __forceinline__ uint64_t walk_mod_quad(int p, int lane, const int32_t *D, const ModP &m) {
    const uint32_t L = 1u << (p - 7);   // a multiple of 4
    int32_t h[R];
    start_rows<R>(h, p, lane, D);
    int32_t da[NA], db[NB];
#pragma unroll
    for (int i = 0; i < NA; ++i) da[i] = D[i];
#pragma unroll
    for (int i = 0; i < NB; ++i) db[i] = D[PM + NA + i];
    double acc = 0.0;   // in [0, p)
    for (uint32_t s = 0;;) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            int32_t a0[NA], a1[NA], b0[NB], b1[NB];
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                a0[i] = h[i];
                a1[i] = h[i] + da[i];
            }
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                b0[i] = h[NA + i];
                b1[i] = h[NA + i] + db[i];
            }
            const double da_ = mod_small<NA>(a0, m) - mod_small<NA>(a1, m) + m.p;   // [1, 2p)
            const double db_ = mod_small<NB>(b0, m) - mod_small<NB>(b1, m) + m.p;
            const double x = red_f(red_f(da_ * db_, m) * mod_rows<R, NA + NB>(h, m), m);
            acc = half ? acc - x : acc + x;   // blocks alternate in sign
            acc = acc < 0.0 ? acc + m.p : (acc >= m.p ? acc - m.p : acc);
            s += 4;
            if (s >= L) {
                const double v = (lane & 1) ? (acc == 0.0 ? 0.0 : m.p - acc) : acc;
                return (uint64_t)v;
            }
            add_rows<R>(h, flip_column(D, s));
        }
    }
}

// per(leaf) modulo p from the lanes' shares of V = (-1)^(p-1) 2^(p-1) per(leaf): the wave's sum,
// times (-1)^(p-1) and the inverse of 2^(p-1) (2^-1 = (q + 1) / 2 for the odd prime q).
__device__ __forceinline__ uint64_t mod_normalise(uint64_t share, int p, const ModP &m) {
    const double V = red_f((double)uni64(wave_sum64(share)), m);   // below 64 p < 2^24
    const double half = (m.p + 1.0) * 0.5;
    double inv = 1.0;
    for (int k = 1; k < p; ++k) inv = red_f(inv * half, m);
    double r = red_f(V * inv, m);
    if ((p - 1) & 1) r = r == 0.0 ? 0.0 : m.p - r;
    return (uint64_t)r;
}

// ------------------------------------------------------------------ per-wave LDS region
// The node being walked lives in one physical mm x mm matrix M (row stride S = dstride(mm))
// with masks of its alive rows and columns: a split marks its deleted row (or column) and the
// merged pair's second line dead and writes the merged line over the pair's first one, so the
// lines keep their relative order (the line order of the node is the physical order of its
// alive lines) and a child costs O(mm) instead of a copy. Per alive row i: rmask[i], the alive
// columns holding a nonzero of row i; per alive column j: cmask[j], the alive rows holding a
// nonzero of column j; rsum[i], the sum of row i over alive columns. Every split node of the
// path keeps an undo record at its order u: its plan, its alive masks, copies of rmask, cmask
// and rsum, and the lines its children overwrite.
__host__ __device__ constexpr int lvl_words(int mm) { return align4(CTL + 5 * mm); }   // see Ctl
// The main kernel's region: M, the leaf tables, the node state, the undo records.
__host__ __device__ constexpr int region_words2(int t, int mm) {
    return mm * dstride(mm) + leaf_table_words() + align4(3 * mm) + 64 + (mm - t) * lvl_words(mm) + SW;
}
// The replay kernel's region: M, tables of every row (stride S), the node state; no records.
__host__ __device__ constexpr int wide_region_words(int mm) {
    return 2 * mm * dstride(mm) + align4(3 * mm) + 64 + SW;
}

struct Region {
    uint32_t *M;                    // mm x S
    int32_t *D;                     // leaf tables (main kernel: leaf_table_words(); replay: mm x S)
    uint32_t *rmask, *cmask, *rsum; // the current node
    uint32_t *rmap, *cmap;          // leaf compaction: alive row / column of each logical index
    uint32_t *lv0;                  // undo record of order t + 1 (main kernel)
    int S, mm, t, lw;
    uint32_t modp = 0;              // modular mode: merged entries reduced modulo this prime
    ModP mp{0.0, 0.0};
    __device__ Region(uint32_t *l, int t_, int mm_, int table_words, uint32_t modp_ = 0)
        : S(dstride(mm_)), mm(mm_), t(t_), lw(lvl_words(mm_)), modp(modp_) {
        if (modp_) mp = ModP{(double)modp_, 1.0 / (double)modp_};
        M = l;
        D = (int32_t *)(l + mm * S);
        rmask = (uint32_t *)(D + table_words);
        cmask = rmask + mm;
        rsum = cmask + mm;
        rmap = rmask + align4(3 * mm);
        cmap = rmap + 32;
        lv0 = cmap + 32;
    }
    __device__ uint32_t *lvl(int u) const { return lv0 + (u - t - 1) * lw; }   // u in t+1 .. mm
    // modular mode: the prime of the job being walked
    __device__ void set_modulus(uint32_t p) {
        modp = p;
        mp = ModP{(double)p, 1.0 / (double)p};
    }
    // a merged entry ca q + cb p (< 2^37) modulo the prime, in FP64 (no integer division)
    __device__ uint32_t reduce(uint64_t v) const { return (uint32_t)red_f((double)v, mp); }
};

// An undo record (order u): the split's weights ca0, cb0, ca1, cb1; one packed word (is_col,
// line, number of pairs, P0, Q0, P1, Q1: 1 + 5 + 2 + 4 x 5 bits); the parent's alive rows and
// columns; the child being walked; then the parent's line masks (rows, then columns), its row
// sums and the lines its two children overwrite.
struct Ctl {
    enum { CA0, CB0, CA1, CB1, PACKED, AR, AC, NEXT };
};
__device__ __forceinline__ uint32_t *sv_msk(const Region &rg, int u) { return rg.lvl(u) + CTL; }
__device__ __forceinline__ uint32_t *sv_rs(const Region &rg, int u) { return rg.lvl(u) + CTL + 2 * rg.mm; }
__device__ __forceinline__ uint32_t *sv_line(const Region &rg, int u, int ch) { return rg.lvl(u) + CTL + (3 + ch) * rg.mm; }
__device__ __forceinline__ uint32_t pk_is_col(uint32_t w) { return w & 1u; }
__device__ __forceinline__ uint32_t pk_line(uint32_t w) { return (w >> 1) & 31u; }
__device__ __forceinline__ uint32_t pk_np(uint32_t w) { return (w >> 6) & 3u; }
__device__ __forceinline__ uint32_t pk_P(uint32_t w, int c) { return (w >> (8 + 10 * c)) & 31u; }
__device__ __forceinline__ uint32_t pk_Q(uint32_t w, int c) { return (w >> (13 + 10 * c)) & 31u; }

// The current node's lines, held in registers: lane i < 32 holds row i (msk: its nonzeros over
// the alive columns, rs: its sum over them), lane 32 + j holds column j (msk: its nonzeros over
// the alive rows). Lanes of dead lines keep stale values that nothing reads.
struct Lines {
    uint32_t msk, rs;
};

// The lines of a node just loaded into the LDS masks (after its wave_sync).
__device__ __forceinline__ Lines lines_from_lds(const Region &rg, int lane) {
    const int k = lane & 31;
    Lines ln;
    ln.msk = k < rg.mm ? (lane < 32 ? rg.rmask[k] : rg.cmask[k]) : 0u;
    ln.rs = lane < 32 && k < rg.mm ? rg.rsum[k] : 0u;
    return ln;
}

// Clears the m x m corner of M; returns the alive mask of m lines.
__device__ __forceinline__ uint32_t clear_node(const Region &rg, int m, int lane) {
    for (int e = lane; e < m * rg.S; e += SW) rg.M[e] = 0;
    if (lane < rg.mm) {
        rg.rmask[lane] = 0;
        rg.cmask[lane] = 0;
        rg.rsum[lane] = 0;
    }
    wave_sync();
    return m >= 32 ? 0xffffffffu : (1u << m) - 1;
}

// Job `job` of a host job table as a dense m x m matrix (Gray columns 0..m-2, then the fixed
// column), with its masks and row sums. Returns m.
__device__ __forceinline__ int load_job(const Region &rg, const JobDesc *jobs, const uint32_t *data, uint32_t job, int lane) {
    const JobDesc jd = jobs[job];
    const int m = (int)uni(jd.m);
    const uint32_t nnz = uni(jd.nnz);
    const uint32_t *blk = data + (size_t)uni(jd.data_off) * HP_DATA_ALIGN;
    const int S = rg.S;
    clear_node(rg, m, lane);
    const uint32_t cs = lane < m ? blk[m + lane] : 0xffffffffu;   // column starts, end at m-1
    for (uint32_t e0 = 0; e0 < nnz; e0 += SW) {
        const uint32_t e = e0 + (uint32_t)lane;
        uint32_t g = 0;   // Gray column of entry e: the last start <= e among columns 1..m-2
        for (int k = 1; k + 1 < m; ++k) g += (uint32_t)__shfl((int)cs, k) <= e;
        if (e < nnz) {
            const uint32_t w = blk[3 * m + e], i = w & 0xffu, b = w >> 9;
            rg.M[i * S + g] = b;
            atomicOr(rg.rmask + i, 1u << g);
            atomicOr(rg.cmask + g, 1u << i);
            atomicAdd(rg.rsum + i, b);
        }
    }
    wave_sync();
    uint32_t bf = 0;
    if (lane < m) {   // fixed column: b_i = base_i + the row's Gray entries
        bf = (uint32_t)((int32_t)blk[lane] + (int32_t)rg.rsum[lane]);
        rg.M[lane * S + m - 1] = bf;
        rg.rsum[lane] += bf;
        if (bf) rg.rmask[lane] |= 1u << (m - 1);
    }
    const uint64_t fixed_rows = __ballot(lane < m && bf != 0);
    if (lane == 0) rg.cmask[m - 1] = (uint32_t)fixed_rows;
    wave_sync();
    return m;
}

// A node of the device expansion (hp_node_words) as a dense matrix, with its masks and row
// sums: lane i reads row i. Returns its order; *bound and *problem receive its header words.
__device__ __forceinline__ int load_node(const Region &rg, const uint32_t *node, int lane, float *bound,
                                         uint32_t *problem) {
    const uint32_t h0 = uni(node[0]);
    const int o = (int)(h0 & 0xffu);
    *bound = __uint_as_float(uni(node[1]));
    *problem = uni(node[2]);
    clear_node(rg, o, lane);
    const uint32_t len = lane < o ? (node[4 + lane / 4] >> (8 * (lane & 3))) & 0xffu : 0u;
    const uint32_t start = wave_scan(len, lane) - len;
    const uint32_t *ent = node + 4 + (o + 3) / 4;
    uint32_t rm = 0, rs = 0;
    for (uint32_t e = 0; e < len; ++e) {
        const uint32_t w = ent[start + e], j = w & 0xffu, v = w >> 8;
        rg.M[lane * rg.S + j] = v;
        rm |= 1u << j;
        rs += v;
        atomicOr(rg.cmask + j, 1u << lane);
    }
    if (lane < o) {
        rg.rmask[lane] = rm;
        rg.rsum[lane] = rs;
    }
    wave_sync();
    return o;
}

// Step 1 of H_per at the current node: (count << 6) | (32 * is_col + index) of the sparsest
// line (rows before columns, then the lowest index; physical order is the node's line order);
// *nz receives that line's nonzero mask.
__device__ __forceinline__ uint32_t sparsest_line(const Lines &ln, uint32_t AR, uint32_t AC, int lane, uint32_t *nz) {
    const bool row = lane < 32 && ((AR >> lane) & 1), col = lane >= 32 && ((AC >> (lane - 32)) & 1);
    const uint32_t cnt = row || col ? (uint32_t)__popc(ln.msk) : 0u;
    uint32_t s;
    const uint32_t w = argmin_lane(cnt, row || col, &s);
    *nz = (uint32_t)__builtin_amdgcn_readlane((int)ln.msk, (int)w);
    return (s << 6) | w;
}

// A split: the line (row or column index), its pairs (positions P, Q and weights ca, cb of
// the merge ca * y_Q + cb * y_P) and their number.
struct Plan {
    uint32_t is_col, line, np;
    uint32_t P[2], Q[2], ca[2], cb[2];
};

// What the plan read for its children, per lane: the entries at Q_c and P_c along the lane's
// own line (rows of a row split, columns of a column split) and, on lanes i < 32, the entry of
// row i on the split line (column splits).
struct PairVals {
    uint32_t q[2], p[2], lv;
};

__device__ __forceinline__ Plan load_plan(const Region &rg, int u) {
    const uint4 w0 = *(const uint4 *)rg.lvl(u);
    const uint32_t pk = uni(rg.lvl(u)[Ctl::PACKED]);
    Plan pl;
    pl.is_col = pk_is_col(pk);
    pl.line = pk_line(pk);
    pl.np = pk_np(pk);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        pl.P[c] = pk_P(pk, c);
        pl.Q[c] = pk_Q(pk, c);
    }
    pl.ca[0] = uni(w0.x);
    pl.cb[0] = uni(w0.y);
    pl.ca[1] = uni(w0.z);
    pl.cb[1] = uni(w0.w);
    return pl;
}

// Pairs of expansion (2) along the line (nonzeros in increasing index order; an odd last one
// with the lowest zero of the line at weight 0). Returns false when a child would break the
// entry or row-sum bound. With `record` (a split of the main walk at order u) the plan, the
// alive masks and the parent's state that the children overwrite go to the undo record.
// COL: the line is a column. Branch-free where it can be: the second pair's entries are read
// even when there is one pair (its positions are then valid, its results unused).
template <bool COL>
__device__ __forceinline__ bool plan_split_t(const Region &rg, uint32_t AR, uint32_t AC, uint32_t s, uint32_t line,
                                            uint32_t nz, const Lines &ln, int lane, Plan &pl, PairVals &pv,
                                            bool record, int u) {
    const int S = rg.S;
    const uint32_t *M = rg.M;
    const uint32_t other = COL ? AR : AC;   // the positions along the line
    pv.lv = lane < 32 && ((other >> lane) & 1) ? (COL ? M[lane * S + line] : M[line * S + lane]) : 0u;
    const uint32_t zero = (uint32_t)__builtin_ctz(~nz & other);
    uint32_t pos[4], val[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {   // bit 31 is never a position: ctz gives 31 once nz is empty
        const uint32_t at = (uint32_t)__builtin_ctz(nz | 0x80000000u);
        nz &= nz - 1;
        pos[k] = (uint32_t)k < s ? at : zero;
        val[k] = (uint32_t)__builtin_amdgcn_readlane((int)pv.lv, (int)pos[k]);
        val[k] = (uint32_t)k < s ? val[k] : 0u;
    }
    const uint32_t np = (s + 1) / 2;
    const int k = lane & 31;
    // the lane's own line takes part in the merge: another alive row (row split) or another
    // alive column (column split)
    const bool mine = COL ? lane >= 32 && ((AC >> k) & 1) && (uint32_t)k != line
                          : lane < 32 && ((AR >> k) & 1) && (uint32_t)k != line;
    bool fail = false;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const uint32_t P = pos[2 * c], Q = pos[2 * c + 1];
        const uint64_t ca = val[2 * c], cb = val[2 * c + 1];
        const bool live = (uint32_t)c < np;
        pv.q[c] = pv.p[c] = 0;
        if (mine) {
            pv.q[c] = COL ? M[Q * S + k] : M[k * S + Q];
            pv.p[c] = COL ? M[P * S + k] : M[k * S + P];
            uint64_t mv = ca * pv.q[c] + cb * pv.p[c];
            if (rg.modp) mv = rg.reduce(mv);
            bool bad = mv >= HP_MAX_ENTRY;
            if (!COL) bad = bad || (uint64_t)ln.rs - pv.q[c] - pv.p[c] + mv >= HP_MAX_ROWSUM;
            fail = fail || (live && bad);
        }
        // the merged row's sum from rows P and Q without the split column (modular mode: every
        // entry stays below p, so every row sum below 2^24, and the bound is not needed)
        if (COL && !rg.modp) {
            const uint64_t rq = (uint32_t)__builtin_amdgcn_readlane((int)ln.rs, (int)Q) -
                                (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)pv.lv, (int)Q);
            const uint64_t rp = (uint32_t)__builtin_amdgcn_readlane((int)ln.rs, (int)P) -
                                (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)pv.lv, (int)P);
            fail = fail || (live && ca * rq + cb * rp >= HP_MAX_ROWSUM);
        }
    }
    if (__ballot(fail) != 0) return false;
    pl.is_col = COL;
    pl.line = line;
    pl.np = np;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        pl.P[c] = pos[2 * c];
        pl.Q[c] = pos[2 * c + 1];
        pl.ca[c] = val[2 * c];
        pl.cb[c] = val[2 * c + 1];
    }
    if (record) {
        uint32_t *ctl = rg.lvl(u);
        if (lane == 0) {
            const uint32_t pk = (uint32_t)COL | line << 1 | np << 6 | pos[0] << 8 | pos[1] << 13 | pos[2] << 18 | pos[3] << 23;
            *(uint4 *)ctl = make_uint4(val[0], val[1], val[2], val[3]);
            *(uint4 *)(ctl + 4) = make_uint4(pk, AR, AC, 0u);
        }
        if (k < rg.mm) {
            sv_msk(rg, u)[(lane >> 5) * rg.mm + k] = ln.msk;
            if (lane < 32) sv_rs(rg, u)[k] = ln.rs;
        }
        if (mine) {   // the lines the children overwrite: the pair's first line, per child
#pragma unroll
            for (int c = 0; c < 2; ++c) sv_line(rg, u, c)[k] = pos[2 * c] < pos[2 * c + 1] ? pv.p[c] : pv.q[c];
        }
        wave_sync();
    }
    return true;
}

__device__ __forceinline__ bool plan_split(const Region &rg, uint32_t AR, uint32_t AC, uint32_t key, uint32_t nz,
                                          const Lines &ln, int lane, Plan &pl, PairVals &pv, bool record, int u) {
    const uint32_t s = key >> 6, line = key & 31;
    return (key >> 5) & 1 ? plan_split_t<true>(rg, AR, AC, s, line, nz, ln, lane, pl, pv, record, u)
                          : plan_split_t<false>(rg, AR, AC, s, line, nz, ln, lane, pl, pv, record, u);
}

// Child `ch` of the current node (plan pl; alive masks AR, AC and the lines ln updated): the
// merged line over the pair's first line, the other line and the split line dead. With `pv`
// the entries the plan read are used, else they are read from M.
template <bool COL>
__device__ __forceinline__ void apply_child_t(const Region &rg, const Plan &pl, int ch, uint32_t &AR, uint32_t &AC,
                                              Lines &ln, const PairVals *pv, int lane) {
    const int S = rg.S;
    uint32_t *M = rg.M;
    const uint32_t line = pl.line;
    const uint32_t P = ch ? pl.P[1] : pl.P[0], Q = ch ? pl.Q[1] : pl.Q[0];
    const uint32_t ca = ch ? pl.ca[1] : pl.ca[0], cb = ch ? pl.cb[1] : pl.cb[0];
    const uint32_t keep = min(P, Q), drop = max(P, Q);
    const uint32_t kb = 1u << keep, db = 1u << drop;
    const int k = lane & 31;
    if (!COL) {   // row `line` deleted; columns P, Q merged into column keep
        const uint32_t AR2 = AR & ~(1u << line), AC2 = AC & ~db;
        const bool row = lane < 32 && ((AR2 >> k) & 1);
        uint32_t mv = 0;
        if (row) {
            const uint32_t mq = pv ? (ch ? pv->q[1] : pv->q[0]) : M[k * S + Q];
            const uint32_t mp = pv ? (ch ? pv->p[1] : pv->p[0]) : M[k * S + P];
            mv = rg.modp ? rg.reduce((uint64_t)ca * mq + (uint64_t)cb * mp) : ca * mq + cb * mp;
            ln.msk = (ln.msk & ~(kb | db)) | (mv ? kb : 0u);
            ln.rs = ln.rs - mq - mp + mv;
            M[k * S + keep] = mv;   // each lane rewrites its own row: no other lane reads it here
        }
        const uint32_t newcol = (uint32_t)__ballot(row && mv != 0);
        if (lane >= 32 && ((AC2 >> k) & 1)) ln.msk = (uint32_t)k == keep ? newcol : ln.msk & ~(1u << line);
        AR = AR2;
        AC = AC2;
    } else {      // column `line` deleted; rows P, Q merged into row keep
        const uint32_t AR2 = AR & ~db, AC2 = AC & ~(1u << line);
        const uint32_t lv = pv ? pv->lv : (lane < 32 && ((AR >> k) & 1) ? M[k * S + line] : 0u);
        const uint32_t rq = (uint32_t)__builtin_amdgcn_readlane((int)ln.rs, (int)Q) -
                            (uint32_t)__builtin_amdgcn_readlane((int)lv, (int)Q);
        const uint32_t rp = (uint32_t)__builtin_amdgcn_readlane((int)ln.rs, (int)P) -
                            (uint32_t)__builtin_amdgcn_readlane((int)lv, (int)P);
        const bool col = lane >= 32 && ((AC2 >> k) & 1);
        uint32_t mv = 0;
        if (col) {
            const uint32_t mq = pv ? (ch ? pv->q[1] : pv->q[0]) : M[Q * S + k];
            const uint32_t mp = pv ? (ch ? pv->p[1] : pv->p[0]) : M[P * S + k];
            mv = rg.modp ? rg.reduce((uint64_t)ca * mq + (uint64_t)cb * mp) : ca * mq + cb * mp;
            ln.msk = (ln.msk & ~(kb | db)) | (mv ? kb : 0u);
            M[keep * S + k] = mv;   // each lane rewrites its own column's entry
        }
        const uint32_t newrow = (uint32_t)(__ballot(col && mv != 0) >> 32);
        // the merged row's sum: from rows P and Q, or (modular mode, entries reduced) the sum
        // of its new entries
        uint32_t krs = ca * rq + cb * rp;
        if (rg.modp) {
            uint32_t part = col ? mv : 0u;
            for (int o = 32; o; o >>= 1) part += (uint32_t)__shfl_xor((int)part, o);
            krs = part;
        }
        if (lane < 32 && ((AR2 >> k) & 1)) {
            const bool kp = (uint32_t)k == keep;
            ln.msk = kp ? newrow : ln.msk & ~(1u << line);
            ln.rs = kp ? krs : ln.rs - lv;
        }
        AR = AR2;
        AC = AC2;
    }
    wave_sync();
}

__device__ __forceinline__ void apply_child(const Region &rg, const Plan &pl, int ch, uint32_t &AR, uint32_t &AC,
                                            Lines &ln, const PairVals *pv, int lane) {
    if (pl.is_col) apply_child_t<true>(rg, pl, ch, AR, AC, ln, pv, lane);
    else apply_child_t<false>(rg, pl, ch, AR, AC, ln, pv, lane);
}

// Back to the state of the split node at order u before child ch was applied: the line child
// ch overwrote and, with `masks`, the node's lines.
__device__ __forceinline__ void restore_node(const Region &rg, int u, int ch, bool masks, Lines &ln, int lane) {
    const uint32_t *ctl = rg.lvl(u);
    const uint32_t pk = uni(ctl[Ctl::PACKED]);
    const uint32_t AR = uni(ctl[Ctl::AR]), AC = uni(ctl[Ctl::AC]);
    const uint32_t is_col = pk_is_col(pk), line = pk_line(pk);
    const uint32_t keep = min(pk_P(pk, ch), pk_Q(pk, ch));
    const int k = lane & 31;
    const bool mine = is_col ? lane >= 32 && ((AC >> k) & 1) && (uint32_t)k != line
                             : lane < 32 && ((AR >> k) & 1) && (uint32_t)k != line;
    if (mine) {
        const uint32_t v = sv_line(rg, u, ch)[k];
        if (is_col) rg.M[keep * rg.S + k] = v;
        else rg.M[k * rg.S + keep] = v;
    }
    if (masks && k < rg.mm) {
        ln.msk = sv_msk(rg, u)[(lane >> 5) * rg.mm + k];
        if (lane < 32) ln.rs = sv_rs(rg, u)[k];
    }
    wave_sync();
}

// The leaf's row and column order: rmap / cmap list the node's alive rows and its alive
// columns but the last (the fixed one, returned in *fx) in physical order; its sparsest Gray
// column c0 (returned; *b its nonzero count, *touched its rows) is moved to Gray column 0 and
// the rows it touches to the front (the product is invariant under both permutations).
__device__ __forceinline__ uint32_t leaf_order(const Region &rg, const Lines &ln, int p, uint32_t AR, uint32_t AC,
                                               int lane, uint32_t *fx, uint32_t *b, uint32_t *touched,
                                               uint32_t *lane_cmk = nullptr) {
    *fx = 31u - (uint32_t)__builtin_clz(AC);   // the fixed (last) column
    // mbcnt: the set bits of a mask below this lane (lanes < 32)
    if (lane < 32 && ((AC >> lane) & 1) && (uint32_t)lane != *fx) rg.cmap[__builtin_amdgcn_mbcnt_lo(AC, 0u)] = (uint32_t)lane;
    if (lane < 32 && ((AR >> lane) & 1)) rg.rmap[__builtin_amdgcn_mbcnt_lo(AR, 0u)] = (uint32_t)lane;
    wave_sync();
    const uint32_t src = lane < p - 1 ? 32u + rg.cmap[lane] : 32u;
    const uint32_t cmk0 = (uint32_t)__shfl((int)ln.msk, (int)src);   // every lane takes part
    const uint32_t cmk = lane < p - 1 ? cmk0 : 0u;
    const uint32_t c0 = argmin_lane((uint32_t)__popc(cmk), lane < p - 1, b);
    *touched = (uint32_t)__builtin_amdgcn_readlane((int)cmk, (int)c0);   // physical rows
    if (lane_cmk) *lane_cmk = cmk;
    return c0;
}

// The main kernel's leaf layout. Gray column 0 is the sparsest column c0 (rows A); for the
// four-step walk Gray column 1 is the sparsest column c1 whose rows B avoid A. Table rows: A,
// then fillers (rows neither column touches) up to pa, then B, fillers up to pa + pb, then the
// other rows, each group in physical order. Without the four-step walk pa = |A| and pb = |B|.
struct LeafPlan {
    uint32_t fx;        // the fixed (last) column
    uint32_t c0, k1;    // c0; the position of c1 after c0 moved to Gray column 0 (1: none)
    uint32_t ta, tb;    // physical rows of A and B
    uint32_t na, nb;    // |A|, |B| (nb = 0: no c1)
    uint32_t pa, pb;    // the groups' sizes in the table
    bool quad;          // the four-step walk applies
};

__device__ __forceinline__ LeafPlan leaf_plan(const Region &rg, const Lines &ln, int p, uint32_t AR, uint32_t AC,
                                              int lane) {
    LeafPlan lp;
    uint32_t cmk;
    lp.c0 = leaf_order(rg, ln, p, AR, AC, lane, &lp.fx, &lp.na, &lp.ta, &cmk);
    const bool cand = lane < p - 1 && (uint32_t)lane != lp.c0 && (cmk & lp.ta) == 0u && cmk != 0u;
    lp.nb = 0;
    lp.tb = 0;
    lp.k1 = 1;
    if (__ballot(cand) != 0 && p >= 9 && lp.na <= 3) {
        uint32_t nb;
        const uint32_t c1 = argmin_lane((uint32_t)__popc(cmk), cand, &nb);
        if (nb <= 3) {
            lp.nb = nb;
            lp.tb = (uint32_t)__builtin_amdgcn_readlane((int)cmk, (int)c1);
            lp.k1 = c1 == 0u ? lp.c0 : c1;
        }
    }
    lp.quad = lp.nb != 0;   // 1 <= |A| <= |B| <= 3 (c0 is the sparsest column)
    lp.pa = lp.quad ? (lp.na <= 2 ? 2u : 3u) : lp.na;
    lp.pb = lp.quad ? (lp.pa == 2u && lp.nb <= 2 ? 2u : 3u) : lp.nb;
    return lp;
}

// Table row of the leaf's physical row r under the plan.
__device__ __forceinline__ int leaf_row4(uint32_t r, const LeafPlan &lp, uint32_t AR) {
    const uint32_t rb = (1u << r) - 1;
    if ((lp.ta >> r) & 1) return __popc(lp.ta & rb);
    if ((lp.tb >> r) & 1) return (int)lp.pa + __popc(lp.tb & rb);
    const int fa = (int)(lp.pa - lp.na), fb = (int)(lp.pb - lp.nb);
    const int o = __popc(AR & ~lp.ta & ~lp.tb & rb);
    if (o < fa) return (int)lp.na + o;
    if (o < fa + fb) return (int)(lp.pa + lp.nb) + (o - fa);
    return (int)(lp.pa + lp.pb) + (o - fa - fb);
}

// The leaf's Gray column behind table column j: c0 moved to 0 (swapped with 0), then c1 to 1.
__device__ __forceinline__ int leaf_col(int j, const LeafPlan &lp) {
    const int c0 = (int)lp.c0, k = (int)lp.k1;
    const int x = j == 1 ? k : (j == k ? 1 : j);
    return x == 0 ? c0 : (x == c0 ? 0 : x);
}

// Table row of the leaf's physical row r: the rows c0 touches first, then the others, each in
// physical order.
__device__ __forceinline__ int leaf_row(uint32_t r, uint32_t touched, uint32_t b, uint32_t AR) {
    const uint32_t rb = (1u << r) - 1;
    return ((touched >> r) & 1) ? __popc(touched & rb) : (int)b + __popc(~touched & AR & rb);
}

// Leaf tables of the main kernel for the current node of order p <= PMAX: D + j PM + i =
// 2 b_ij for Gray column j, D + TNEG + j PM + i its negative, D + 2 TNEG + i = base_i =
// 2 b_{i,p-1} - R_i (rows p..PM-1: deltas 0, base 1, so f = 1), rows and columns laid out by
// the leaf plan, which it returns (Gray column 0's rows and count; column 1 of the four-step
// walk). Needs p >= 2.
__device__ __forceinline__ LeafPlan leaf_tables(const Region &rg, const Lines &ln, int p, uint32_t AR, uint32_t AC,
                                                int lane) {
    const LeafPlan lp = leaf_plan(rg, ln, p, AR, AC, lane);
    // lane = logical row i (its table row computed once) and a quarter of the Gray columns
    const int i = lane & (PM - 1), jq = lane >> 4;
    const uint32_t r = i < p ? rg.rmap[i] : 0u;
    const uint32_t rsr = (uint32_t)__shfl((int)ln.rs, (int)r);   // every lane takes part
    const int pos = i < p ? leaf_row4(r, lp, AR) : i;            // padding rows keep their place
    const uint32_t *Mr = rg.M + r * rg.S;
    for (int j = jq; j < p - 1; j += SW / PM) {
        const int32_t v = i < p ? 2 * (int32_t)Mr[rg.cmap[leaf_col(j, lp)]] : 0;
        rg.D[j * PM + pos] = v;
        rg.D[TNEG + j * PM + pos] = -v;
    }
    if (jq == 0) rg.D[2 * TNEG + pos] = i < p ? 2 * (int32_t)Mr[lp.fx] - (int32_t)rsr : 1;
    wave_sync();
    return lp;
}

// The replay kernel's tables (rows of stride S, every row of the node): D + j S + i = 2 b_ij,
// base at D + (mm - 1) S. Returns nothing; the replay walks every step.
__device__ __forceinline__ void leaf_tables_wide(const Region &rg, const Lines &ln, int p, uint32_t AR, uint32_t AC,
                                                 int lane) {
    uint32_t fx, b, touched;
    const uint32_t c0 = leaf_order(rg, ln, p, AR, AC, lane, &fx, &b, &touched);
    const uint32_t rsr = (uint32_t)__shfl((int)ln.rs, lane < p ? (int)rg.rmap[lane] : 0);
    const int S = rg.S;
    int32_t *base = rg.D + (rg.mm - 1) * S;
    for (int e = lane; e < (p - 1) * S; e += SW) {
        const int j = e / S, i = e - j * S;
        if (i < p) {
            const uint32_t r = rg.rmap[i];
            const int g = j == 0 ? (int)c0 : (j == (int)c0 ? 0 : j);
            rg.D[j * S + leaf_row(r, touched, b, AR)] = 2 * (int32_t)rg.M[r * S + rg.cmap[g]];
        } else {
            rg.D[e] = 0;
        }
    }
    if (lane < S) {
        if (lane < p) {
            const uint32_t r = rg.rmap[lane];
            base[leaf_row(r, touched, b, AR)] = 2 * (int32_t)rg.M[r * S + fx] - (int32_t)rsr;
        } else {
            base[lane] = 1;
        }
    }
    wave_sync();
}

// This lane's share of V = (-1)^(p-1) 2^(p-1) per(leaf) modulo 2^64 for a leaf of order
// 7 <= p <= PMAX.
__device__ __forceinline__ uint64_t eval_leaf(const Region &rg, const Lines &ln, int p, uint32_t AR, uint32_t AC,
                                              int lane) {
    const LeafPlan lp = leaf_tables(rg, ln, p, AR, AC, lane);
    const uint32_t b = lp.na;
    uint64_t v;
    if (lp.quad) {   // p >= 9
        const uint32_t k = lp.pa == 2 ? (lp.pb == 2 ? 0u : 1u) : 2u;
        if (p <= 12) v = k == 0 ? walk_quad<12, 2, 2>(p, lane, rg.D)
                               : (k == 1 ? walk_quad<12, 2, 3>(p, lane, rg.D) : walk_quad<12, 3, 3>(p, lane, rg.D));
        else v = k == 0 ? walk_quad<16, 2, 2>(p, lane, rg.D)
                        : (k == 1 ? walk_quad<16, 2, 3>(p, lane, rg.D) : walk_quad<16, 3, 3>(p, lane, rg.D));
    } else if (p >= 8 && p <= 12 && b <= 2) v = walk_paired<12, 2>(p, lane, rg.D);
    else if (p >= 8 && p <= 12 && b <= 4) v = walk_paired<12, 4>(p, lane, rg.D);
    else if (p <= 12) v = walk_plain<12>(p, lane, rg.D);
    else if (b <= 2) v = walk_paired<16, 2>(p, lane, rg.D);
    else if (b <= 4) v = walk_paired<16, 4>(p, lane, rg.D);
    else v = walk_plain<16>(p, lane, rg.D);
    wave_sync();   // the tables are rewritten by the next leaf
    return v;
}

// Proven log2 upper bounds of per(node): the product of its row sums, and of its column sums.
__device__ __forceinline__ float rowsum_log2(const Lines &ln, uint32_t AR, int lane) {
    const float x = lane < 32 && ((AR >> lane) & 1) ? __log2f((float)ln.rs) : 0.0f;   // < 2^24: exact
    return wave_sumf(x) + 1e-3f;   // margin for the hardware logarithm and the float sum
}
__device__ __forceinline__ float colsum_log2(const Region &rg, uint32_t AR, uint32_t AC, int lane) {
    float x = 0.0f;
    if (lane < 32 && ((AC >> lane) & 1)) {
        uint32_t cs = 0;   // below 24 * 2^22 < 2^27: the float is within one part in 2^24
        for (uint32_t rows = AR; rows; rows &= rows - 1) cs += rg.M[(uint32_t)__builtin_ctz(rows) * rg.S + lane];
        x = __log2f((float)cs) + 1e-6f;
    }
    return wave_sumf(x) + 1e-3f;
}

// per(leaf) from its wave-summed V modulo 2^64: (-1)^(p-1) V / 2^(p-1) after the checks that
// the bound guarantees (non-negative, divisible). *bad is set when a check fails.
__device__ __forceinline__ uint64_t normalise64(uint64_t V, int p, bool *bad) {
    const int sh = p - 1;
    if (sh & 1) V = (uint64_t)0 - V;
    const bool ok = (int64_t)V >= 0 && (sh == 0 || (V & ((1ull << sh) - 1)) == 0);
    *bad = !ok;
    return ok ? V >> sh : 0;
}

__device__ __forceinline__ u128 normalise128(u128 V, int p, bool *bad) {
    const int sh = p - 1;
    if (sh & 1) V = (u128)0 - V;
    const bool ok = (V >> 127) == 0 && (sh == 0 || (V & (((u128)1 << sh) - 1)) == 0);
    *bad = !ok;
    return ok ? V >> sh : 0;
}

// Adds v (a 128-bit per value) as 32-bit limbs into four 64-bit limb sums.
__device__ __forceinline__ void add_limbs(unsigned long long *l, u128 v) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const unsigned long long x = (uint32_t)(v >> (32 * k));
        if (x) atomicAdd(l + k, x);
    }
}

// A deferred leaf: the job, the leaf's order and the child index taken at every order above it
// (bit m - o for the split at order o).
struct WideLeaf {
    uint32_t job;
    uint32_t order_path;   // order | path << 8
};

}  // namespace

// Arguments of the two kernels (shared by both job sources).
struct SplitArgs {
    const JobDesc *jobs;          // host job table (node source: null)
    const uint32_t *data;
    const float *job_bound;       // per host job: its proven log2 bound (rounded up)
    const uint32_t *nodes;        // device expansion's nodes (host source: null)
    const uint64_t *node_off;     // word offset of every node
    const uint32_t *queue;        // host source: job ids in queue order
    uint32_t n;                   // jobs in the queue, or nodes
    uint32_t njobs;               // host source: size of the job table
    int t, s_leaf, mm;
    unsigned long long *head;     // cleared queue counter
    JobAcc *accs;                 // per-job values (nullable for nodes)
    ProbAcc *probs;               // per-problem sums (nodes only)
    unsigned long long *stats;    // 8 counters, cleared
    WideLeaf *wide;
    uint32_t wide_cap;
    unsigned long long *cycles;   // nullable
    const uint32_t *modps;        // nullptr: exact; else per problem a prime below 2^18: per(B) modulo it
};

namespace {

// The job's dense matrix in its top slot, its bound and its problem; returns its order.
template <bool NODES>
__device__ __forceinline__ int load_source(const Region &rg, const SplitArgs &a, uint32_t job, int lane,
                                           float *jb, uint32_t *problem) {
    if constexpr (NODES) {
        return load_node(rg, a.nodes + uni64(a.node_off[job]), lane, jb, problem);
    } else {
        *jb = __uint_as_float(uni(__float_as_uint(a.job_bound[job])));
        *problem = 0;
        return load_job(rg, a.jobs, a.data, job, lane);
    }
}

// Four waves per SIMD: the register budget drops from 143 to 128 VGPRs (a few values of the
// outer loop go to scratch around the leaf walk) and the latency-bound split steps get a third
// more waves to interleave (measured 17 % faster on the order-20 jobs of the cubic graphs on
// 60 vertices at t = 12).
template <bool NODES, bool MOD>
__global__ __launch_bounds__(SW) __attribute__((amdgpu_waves_per_eu(4))) void hper_split(SplitArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    const int lane = threadIdx.x;
    Region rg(lds, a.t, a.mm, leaf_table_words());
    uint64_t n_leaves = 0, n_terms = 0, n_splits = 0, n_stops = 0, n_bad = 0, n_wide = 0;
    u128 pacc = 0;            // this wave's sum for problem pcur (nodes)
    uint32_t pcur = 0xffffffffu;
    for (;;) {
        const unsigned long long got = atomicAdd(a.head, lane == 0 ? 1ull : 0ull);
        const uint64_t qi = uni64(got);
        if (qi >= a.n) break;
        const uint32_t job = NODES ? (uint32_t)qi : uni(a.queue[qi]);
        const uint64_t t0 = (uint64_t)clock64();
        float jb;
        uint32_t problem;
        const int m0 = load_source<NODES>(rg, a, job, lane, &jb, &problem);
        if constexpr (MOD) rg.set_modulus(uni(a.modps[problem]));   // the job's problem's prime
        uint32_t AR = (1u << m0) - 1, AC = AR;   // alive rows and columns of the current node
        Lines ln = lines_from_lds(rg, lane);
        u128 acc = 0;   // per(B): the sum of the normalised leaves (wave-uniform)
        int o = m0;
        Plan pl;
        PairVals pv;
        for (;;) {
            uint32_t nz;
            const uint32_t key = sparsest_line(ln, AR, AC, lane, &nz);
            const uint32_t s = key >> 6;
            if (s != 0) {
                const bool leaf = o <= a.t || o <= 2 || (int)s >= a.s_leaf || s > 4;
                if (!leaf) {
                    if (plan_split(rg, AR, AC, key, nz, ln, lane, pl, pv, true, o)) {
                        apply_child(rg, pl, 0, AR, AC, ln, &pv, lane);
                        ++n_splits;
                        --o;
                        continue;
                    }
                    ++n_stops;   // refused by the entry bounds: evaluated whole
                }
                ++n_leaves;
                n_terms += 1ull << (o - 1);
                // exact modulo 2^64 when per(leaf) 2^(o-1) < 2^63 (bound: the job's, or the
                // leaf's product of row sums); modular mode: every leaf up to order 16 here
                bool ok64 = MOD;
                if (!ok64) ok64 = fminf(jb, rowsum_log2(ln, AR, lane)) + (float)o <= 62.5f;
                if (!ok64 && o <= PMAX) ok64 = colsum_log2(rg, AR, AC, lane) + (float)o <= 62.5f;
                if (MOD && o <= PMAX) {
                    const LeafPlan lp = leaf_tables(rg, ln, o, AR, AC, lane);
                    uint64_t share;
                    if (lp.quad) {
                        const uint32_t k = lp.pa == 2 ? (lp.pb == 2 ? 0u : 1u) : 2u;
                        if (o <= 12)
                            share = k == 0 ? walk_mod_quad<12, 2, 2>(o, lane, rg.D, rg.mp)
                                           : (k == 1 ? walk_mod_quad<12, 2, 3>(o, lane, rg.D, rg.mp)
                                                     : walk_mod_quad<12, 3, 3>(o, lane, rg.D, rg.mp));
                        else
                            share = k == 0 ? walk_mod_quad<16, 2, 2>(o, lane, rg.D, rg.mp)
                                           : (k == 1 ? walk_mod_quad<16, 2, 3>(o, lane, rg.D, rg.mp)
                                                     : walk_mod_quad<16, 3, 3>(o, lane, rg.D, rg.mp));
                    } else {
                        share = o <= 12 ? walk_mod<12>(o, lane, rg.D, rg.mp) : walk_mod<16>(o, lane, rg.D, rg.mp);
                    }
                    wave_sync();   // the tables are rewritten by the next leaf
                    acc += mod_normalise(share, o, rg.mp);
                    if (acc >= (u128)rg.modp) acc -= rg.modp;
                } else if (ok64 && o <= PMAX) {
                    bool bad;
                    const uint64_t per = normalise64(uni64(wave_sum64(eval_leaf(rg, ln, o, AR, AC, lane))), o, &bad);
                    n_bad += bad;
                    acc += per;
                } else {   // replayed by the second kernel in 128-bit arithmetic
                    ++n_wide;
                    uint32_t path = 0;
                    for (int u = o + 1; u <= m0; ++u) path |= uni(rg.lvl(u)[Ctl::NEXT]) << (m0 - u);
                    if (lane == 0) {
                        const unsigned long long w = atomicAdd(a.stats + 4, 1ull);
                        if (w < a.wide_cap) a.wide[w] = WideLeaf{job, (uint32_t)o | (path << 8)};
                        else atomicAdd(a.stats + 5, 1ull);   // reported as an error
                    }
                }
            }
            // back up to the nearest split node of the path with a child left, undoing the
            // lines the children on the way overwrote (the deepest first)
            int up = o + 1;
            for (; up <= m0; ++up) {
                uint32_t *ctl = rg.lvl(up);
                const uint32_t cur = uni(ctl[Ctl::NEXT]), nx = cur + 1;
                if (nx < pk_np(uni(ctl[Ctl::PACKED]))) {
                    restore_node(rg, up, (int)cur, true, ln, lane);
                    AR = uni(ctl[Ctl::AR]);
                    AC = uni(ctl[Ctl::AC]);
                    if (lane == 0) ctl[Ctl::NEXT] = nx;
                    apply_child(rg, load_plan(rg, up), (int)nx, AR, AC, ln, nullptr, lane);
                    break;
                }
                restore_node(rg, up, (int)cur, false, ln, lane);
            }
            if (up > m0) break;
            o = up - 1;
        }
        if (lane == 0) {
            if (a.accs) {
                JobAcc *ja = a.accs + job;
#pragma unroll
                for (int k = 0; k < 4; ++k) ja->l[k] = (uint32_t)(acc >> (32 * k));
                ja->flag = HP_ACC_NORMALISED;
            }
            if (a.cycles) a.cycles[job] = (unsigned long long)((uint64_t)clock64() - t0);
        }
        if constexpr (NODES) {
            if (problem != pcur) {
                if (lane == 0 && pcur != 0xffffffffu) add_limbs(a.probs[pcur].lim, pacc);
                pcur = problem;
                pacc = 0;
            }
            pacc += acc;
        }
    }
    if (lane == 0) {
        if (NODES && pcur != 0xffffffffu) add_limbs(a.probs[pcur].lim, pacc);
        atomicAdd(a.stats + 0, (unsigned long long)n_leaves);
        atomicAdd(a.stats + 1, (unsigned long long)n_terms);
        atomicAdd(a.stats + 2, (unsigned long long)n_splits);
        atomicAdd(a.stats + 3, (unsigned long long)n_stops);
        if (n_bad) atomicAdd(a.stats + 6, (unsigned long long)n_bad);
        if (n_wide) atomicAdd(a.stats + 7, (unsigned long long)n_wide);
    }
}

// The deferred leaves: each wave replays one leaf's path from its job's matrix (the same
// line choices and pairs), evaluates the leaf modulo 2^128 and adds its normalised value to
// the job (and, for nodes, to the problem).
template <bool NODES, bool MOD>
__global__ __launch_bounds__(SW) void hper_split_wide(SplitArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    const int lane = threadIdx.x;
    Region rg(lds, a.t, a.mm, a.mm * dstride(a.mm));
    const uint64_t n = min((uint64_t)a.stats[4], (uint64_t)a.wide_cap);
    for (uint64_t w = blockIdx.x; w < n; w += gridDim.x) {
        const WideLeaf wl = a.wide[w];
        const uint32_t job = uni(wl.job), op = uni(wl.order_path);
        const int p = (int)(op & 0xffu);
        const uint32_t path = op >> 8;
        if (job >= (NODES ? a.n : a.njobs)) continue;
        float jb;
        uint32_t problem;
        const int m0 = load_source<NODES>(rg, a, job, lane, &jb, &problem);
        if constexpr (MOD) rg.set_modulus(uni(a.modps[problem]));
        if (p < 7 || p > m0 || m0 > a.mm) continue;
        uint32_t AR = (1u << m0) - 1, AC = AR;
        Lines ln = lines_from_lds(rg, lane);
        Plan pl;
        PairVals pv;
        for (int o = m0; o > p; --o) {
            uint32_t nz;
            const uint32_t key = sparsest_line(ln, AR, AC, lane, &nz);
            if (!plan_split(rg, AR, AC, key, nz, ln, lane, pl, pv, false, o)) break;   // not reached:
            apply_child(rg, pl, (int)((path >> (m0 - o)) & 1), AR, AC, ln, &pv, lane);   // the first pass split here
        }
        leaf_tables_wide(rg, ln, p, AR, AC, lane);
        const int32_t *base = rg.D + (rg.mm - 1) * rg.S;
        bool bad = false;
        u128 per;
        if (MOD) {   // modular mode: the leaf's residue
            const uint64_t share = rg.S == 20 ? walk_mod_wide<20>(p, lane, rg.D, base, rg.S, rg.mp)
                                              : walk_mod_wide<SMAX>(p, lane, rg.D, base, rg.S, rg.mp);
            per = mod_normalise(share, p, rg.mp);
        } else {
            u128 v;   // rows padded to the table's stride (20 or 24), never beyond it
            if (rg.S == 20) v = walk_plain128<20>(p, lane, rg.D, base, rg.S);
            else v = walk_plain128<SMAX>(p, lane, rg.D, base, rg.S);
            per = normalise128(wave_sum128(v), p, &bad);
        }
        if (lane == 0) {
            if (bad) atomicAdd(a.stats + 6, 1ull);
            if (a.accs) add_limbs(a.accs[job].l, per);
            if (NODES) add_limbs(a.probs[problem].lim, per);
        }
        wave_sync();
    }
}

}  // namespace

size_t split_lds_bytes(int t, int mm) { return (size_t)region_words2(t, mm) * sizeof(uint32_t); }
static size_t wide_lds_bytes(int mm) { return (size_t)wide_region_words(mm) * sizeof(uint32_t); }
size_t split_wide_bytes(uint64_t entries) { return (size_t)(entries ? entries : 1) * sizeof(WideLeaf); }

static hipError_t resident_grid(const void *fn, size_t lds, uint64_t *grid) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, SW, lds);
    if (e != hipSuccess) return e;
    *grid = (uint64_t)cus * (uint64_t)(per_cu > 0 ? per_cu : 1);
    return hipSuccess;
}

template <bool NODES, bool MOD>
static hipError_t launch_split_kernels(const SplitArgs &a, hipStream_t s) {
    const size_t lds = split_lds_bytes(a.t, a.mm);
    uint64_t grid = 0;
    hipError_t e = resident_grid((const void *)hper_split<NODES, MOD>, lds, &grid);
    if (e != hipSuccess) return e;
    if (grid > a.n) grid = a.n;
    hipLaunchKernelGGL((hper_split<NODES, MOD>), dim3((uint32_t)grid), dim3(SW), lds, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t wlds = wide_lds_bytes(a.mm);
    e = resident_grid((const void *)hper_split_wide<NODES, MOD>, wlds, &grid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((hper_split_wide<NODES, MOD>), dim3((uint32_t)grid), dim3(SW), wlds, s, a);
    return hipGetLastError();
}

template <bool NODES>
static hipError_t launch_split_pair(const SplitArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    if (a.t < HP_SPLIT_MIN_T || a.t >= HP_SPLIT_MAX_M || a.mm <= a.t || a.mm > HP_SPLIT_MAX_M) return hipErrorInvalidValue;
    if (a.modps) {   // the modular kernels exist for the device expansion's nodes only
        if (!NODES) return hipErrorInvalidValue;
        return launch_split_kernels<true, true>(a, s);
    }
    return launch_split_kernels<NODES, false>(a, s);
}

int split_grid(int t, int mm) {
    uint64_t grid = 0;
    if (resident_grid((const void *)hper_split<false, false>, split_lds_bytes(t, mm), &grid) != hipSuccess) return 0;
    return (int)grid;
}

hipError_t launch_split_jobs(const JobDesc *jobs, const uint32_t *data, const float *job_bound, const uint32_t *queue,
                             uint32_t n, uint32_t njobs, int t, int mm, int s_leaf, unsigned long long *head,
                             JobAcc *accs, unsigned long long *stats, void *wide, uint64_t wide_entries,
                             unsigned long long *cycles, hipStream_t s) {
    SplitArgs a{};
    a.jobs = jobs;
    a.data = data;
    a.job_bound = job_bound;
    a.queue = queue;
    a.n = n;
    a.njobs = njobs;
    a.t = t;
    a.s_leaf = s_leaf;
    a.mm = mm;
    a.head = head;
    a.accs = accs;
    a.stats = stats;
    a.wide = (WideLeaf *)wide;
    a.wide_cap = (uint32_t)(wide_entries < 0xffffffffull ? wide_entries : 0xffffffffull);
    a.cycles = cycles;
    return launch_split_pair<false>(a, s);
}

hipError_t launch_split_nodes(const uint32_t *nodes, const uint64_t *node_off, uint32_t n, int t, int mm, int s_leaf,
                              unsigned long long *head, JobAcc *accs, ProbAcc *probs, unsigned long long *stats,
                              void *wide, uint64_t wide_entries, const uint32_t *modps, hipStream_t s) {
    SplitArgs a{};
    a.nodes = nodes;
    a.node_off = node_off;
    a.n = n;
    a.njobs = n;
    a.t = t;
    a.s_leaf = s_leaf;
    a.mm = mm;
    a.head = head;
    a.accs = accs;
    a.probs = probs;
    a.stats = stats;
    a.wide = (WideLeaf *)wide;
    a.wide_cap = (uint32_t)(wide_entries < 0xffffffffull ? wide_entries : 0xffffffffull);
    a.modps = modps;
    return launch_split_pair<true>(a, s);
}

}  // namespace hp
