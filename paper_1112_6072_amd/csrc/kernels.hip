// HIP kernels of libhperm for gfx950 (MI355X): R-NW Gray-code evaluation of jobs (a
// persistent queue kernel and a one-launch-per-job kernel sharing one inner loop), the
// KKLLL estimator in FP32, and a fill kernel.
//
// The file is compiled once per HP_PART so that the object files build in parallel:
// HP_PART = 0 holds the estimator and the fill kernel, HP_PART = 1, 2, 3 the R-NW kernels
// of the W64, W128 and residue rings.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hperm_internal.h"
#include "kernels.h"

#ifndef HP_PART
#error "compile with -DHP_PART=0..3"
#endif

namespace {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;   // 4 waves; every wave works on its own item

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
// x as a signed 24-bit value (its bits 24..31 replaced by copies of bit 23): a product of two
// such values compiles to the full-rate 24-bit multiplier. Only for values known to fit.
__device__ __forceinline__ int s24(int x) { return (int)((uint32_t)x << 8) >> 8; }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t x, int mask) {
    uint32_t lo = __shfl_xor((int)(uint32_t)x, mask, WAVE);
    uint32_t hi = __shfl_xor((int)(uint32_t)(x >> 32), mask, WAVE);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
#pragma unroll
    for (int mask = 32; mask >= 1; mask >>= 1) x += shfl_xor64(x, mask);
    return x;
}

__device__ __forceinline__ JobDesc load_job(const JobDesc *jobs, uint32_t j) {
    const uint32_t *p = reinterpret_cast<const uint32_t *>(jobs + j);
    const uint32_t a = uni(p[0]), b = uni(p[1]), c = uni(p[2]), d = uni(p[3]);
    JobDesc jd;
    jd.data_off = a;
    jd.m = (uint8_t)(b & 0xff);
    jd.arith = (uint8_t)((b >> 8) & 0xff);
    jd.chunk_log2 = (uint8_t)((b >> 16) & 0xff);
    jd.flags = (uint8_t)(b >> 24);
    jd.nnz = c;
    jd.problem = d;
    return jd;
}

// x mod p for p = 2^61 - C (residue ring and Step 4 normalisation).
template <uint64_t C>
__device__ __forceinline__ uint64_t mod61(unsigned __int128 x) {
    constexpr uint64_t P = (1ull << 61) - C;
    // x < 2^122: fold 2^61 = C twice (the second fold leaves less than 2P), then subtract
    uint64_t lo = (uint64_t)x & ((1ull << 61) - 1);
    unsigned __int128 hi = x >> 61;
    unsigned __int128 y = (unsigned __int128)lo + hi * C;
    lo = (uint64_t)y & ((1ull << 61) - 1);
    uint64_t h2 = (uint64_t)(y >> 61);
    uint64_t z = lo + h2 * C;   // y < 2^68, so h2 < 2^7 and z < 2P
    return z >= P ? z - P : z;
}
template <uint64_t C>
__device__ __forceinline__ uint64_t mulmod_full(uint64_t a, uint64_t b) {
    return mod61<C>((unsigned __int128)a * b);
}
#if HP_PART >= 1
// ------------------------------------------------------------------------ rings
// A ring multiplies a non-negative product by |f_i| (unsigned, below 2^24) and adds or
// subtracts the product into a lane accumulator. The sign of a term is tracked apart (the
// parity of the negative factors and the Gray sign (-1)^k) and arrives as a mask: all ones
// for a negative term, zero for a positive one.

// pair_mul(s, d): s times the signed integer d (|d| < 2^74) in the ring; the paired walk's
// sum of two terms is S_b * X. Small holds X exactly (below 2^74) in the wide rings and modulo
// 2^64 in the 64-bit one, which is all that ring needs; USmall is its unsigned twin, in which
// the wrapping arithmetic is done.
struct RingW64 {
    struct P { uint64_t v; };
    using Small = int64_t;
    using USmall = uint64_t;
    static constexpr bool kFourStep = true;   // the four-step walk's block sums wrap modulo 2^64
    __device__ static P pair_mul(const P &s, Small d) { return {s.v * (uint64_t)d}; }
    // -p = (p xor ~0) + 1: the accumulator adds p xor mask and counts the +1s apart
    struct Acc { uint64_t v; uint32_t n; };
    __device__ static P one() { return {1}; }
    __device__ static void mul(P &p, uint32_t u) {
        // low word times u as a 64-bit product; high word times u modulo 2^32 as a separate
        // multiply (kept out of a fused multiply-add, whose 64-bit addend needs a register
        // pair and extra moves)
        const uint64_t lo = (uint64_t)(uint32_t)p.v * u;
        uint32_t hi;
        asm volatile("v_mul_lo_u32 %0, %1, %2" : "=v"(hi) : "v"((uint32_t)(p.v >> 32)), "v"(u));
        p.v = lo + ((uint64_t)hi << 32);
    }
    __device__ static Acc acc_zero() { return {0, 0}; }
    __device__ static void acc(Acc &a, const P &p, uint32_t mask) {
        a.v += p.v ^ (((uint64_t)mask << 32) | mask);
        a.n -= mask;
    }
    __device__ static void flush(const Acc &a, JobAcc *dst, int lane) {
        const uint64_t s = wave_sum64(a.v + a.n);
        if (lane == 0) atomicAdd(&dst->l[0], (unsigned long long)s);
    }
};

struct RingW128 {
    static constexpr bool kFourStep = false;
    struct P { uint32_t x0, x1, x2, x3; };
    using Small = __int128;
    using USmall = unsigned __int128;
    __device__ static P pair_mul(const P &s, Small d) {
        const unsigned __int128 v = (((unsigned __int128)s.x3 << 96) | ((unsigned __int128)s.x2 << 64) |
                                     ((unsigned __int128)s.x1 << 32) | s.x0) * (unsigned __int128)d;
        return {(uint32_t)v, (uint32_t)(v >> 32), (uint32_t)(v >> 64), (uint32_t)(v >> 96)};
    }
    // The accumulator keeps four independent 64-bit sums of the 32-bit limbs of (p xor mask)
    // (no carry chain between limbs per term; a lane adds at most 2^12 terms, so each sum
    // stays below 2^44) and the count of the +1s of the negations.
    struct Acc { uint64_t s0, s1, s2, s3; uint32_t n; };
    __device__ static P one() { return {1, 0, 0, 0}; }
    __device__ static void mul(P &p, uint32_t u) {
        const uint64_t t0 = (uint64_t)p.x0 * u;
        const uint64_t t1 = (uint64_t)p.x1 * u + (t0 >> 32);
        const uint64_t t2 = (uint64_t)p.x2 * u + (t1 >> 32);
        const uint32_t t3 = p.x3 * u + (uint32_t)(t2 >> 32);
        p = {(uint32_t)t0, (uint32_t)t1, (uint32_t)t2, t3};
    }
    __device__ static Acc acc_zero() { return {0, 0, 0, 0, 0}; }
    __device__ static void acc(Acc &a, const P &p, uint32_t mask) {
        a.s0 += p.x0 ^ mask;
        a.s1 += p.x1 ^ mask;
        a.s2 += p.x2 ^ mask;
        a.s3 += p.x3 ^ mask;
        a.n -= mask;
    }
    __device__ static void flush(const Acc &a, JobAcc *dst, int lane) {
        // the lane's value sum_k s_k 2^(32k) + n (mod 2^128), renormalised into 32-bit limbs
        const unsigned __int128 v = (unsigned __int128)a.s0 + ((unsigned __int128)a.s1 << 32) +
                                    ((unsigned __int128)a.s2 << 64) + ((unsigned __int128)a.s3 << 96) + a.n;
        const uint64_t s0 = wave_sum64((uint32_t)v), s1 = wave_sum64((uint32_t)(v >> 32));
        const uint64_t s2 = wave_sum64((uint32_t)(v >> 64)), s3 = wave_sum64((uint32_t)(v >> 96));
        if (lane == 0) {
            atomicAdd(&dst->l[0], (unsigned long long)s0);
            atomicAdd(&dst->l[1], (unsigned long long)s1);
            atomicAdd(&dst->l[2], (unsigned long long)s2);
            atomicAdd(&dst->l[3], (unsigned long long)s3);
        }
    }
};

// Residues modulo p_k = 2^61 - c_k. A product r * u with r < p and u < 2^24 is below 2^85;
// 2^61 = c_k (mod p_k) folds it to lo + c_k * hi < 2 p_k, then one conditional subtraction.
template <uint64_t C>
__device__ __forceinline__ uint64_t mulmod61(uint64_t r, uint32_t u) {
    constexpr uint64_t P = (1ull << 61) - C;
    const unsigned __int128 x = (unsigned __int128)r * u;
    const uint64_t lo = (uint64_t)x & ((1ull << 61) - 1);
    const uint64_t hi = (uint64_t)(x >> 61);
    uint64_t s = lo + C * hi;
    return s >= P ? s - P : s;
}
template <uint64_t C>
__device__ __forceinline__ uint64_t addmod61(uint64_t a, uint64_t b, uint32_t neg) {
    constexpr uint64_t P = (1ull << 61) - C;
    if (neg) return a >= b ? a - b : a + P - b;
    const uint64_t s = a + b;
    return s >= P ? s - P : s;
}

template <uint64_t C>
__device__ __forceinline__ uint64_t mulmod_signed(uint64_t r, __int128 d) {
    constexpr uint64_t P = (1ull << 61) - C;
    const bool neg = d < 0;
    uint64_t a = mod61<C>((unsigned __int128)(neg ? -d : d));
    if (neg && a) a = P - a;
    return mulmod_full<C>(r, a);
}

struct RingRes {
    static constexpr bool kFourStep = false;
    struct P { uint64_t r0, r1, r2; };
    using Acc = P;
    using Small = __int128;
    using USmall = unsigned __int128;
    __device__ static P pair_mul(const P &s, Small d) {
        return {mulmod_signed<HP_C0>(s.r0, d), mulmod_signed<HP_C1>(s.r1, d), mulmod_signed<HP_C2>(s.r2, d)};
    }
    __device__ static P one() { return {1, 1, 1}; }
    __device__ static void mul(P &p, uint32_t u) {
        p.r0 = mulmod61<HP_C0>(p.r0, u);
        p.r1 = mulmod61<HP_C1>(p.r1, u);
        p.r2 = mulmod61<HP_C2>(p.r2, u);
    }
    __device__ static Acc acc_zero() { return {0, 0, 0}; }
    __device__ static void acc(Acc &a, const P &p, uint32_t mask) {
        const uint32_t neg = mask & 1u;
        a.r0 = addmod61<HP_C0>(a.r0, p.r0, neg);
        a.r1 = addmod61<HP_C1>(a.r1, p.r1, neg);
        a.r2 = addmod61<HP_C2>(a.r2, p.r2, neg);
    }
    __device__ static void flush(const Acc &a, JobAcc *dst, int lane) {
        const uint64_t v[3] = {a.r0, a.r1, a.r2};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint64_t lo = wave_sum64(v[k] & 0xffffffffull);
            const uint64_t hi = wave_sum64(v[k] >> 32);
            if (lane == 0) {
                atomicAdd(&dst->l[2 * k], (unsigned long long)lo);
                atomicAdd(&dst->l[2 * k + 1], (unsigned long long)hi);
            }
        }
    }
};

// ------------------------------------------------------------------------ R-NW work item
// One work item is 64 consecutive lane chunks of one job: lane l covers the Gray indices
// [zL, zL + L) of chunk z = item * 64 + l, L = 2^c. An even chunk is walked forwards from
// k = zL, an odd one backwards from k = zL + L - 1. For c >= 1 the reflected Gray code makes
// the odd chunk's walk the even chunk's walk with Gray bit c set: at step t both have the
// low c Gray bits gray(t), so the column flipped after step t is j = ctz(t + 1) and its
// direction (+1 when bit j + 1 of t + 1 is 0) are the same in every lane, for every j < c.
// The lanes differ only in the Gray bits c and up of their first index, which fix their
// starting row values, and in the sign (-1)^k of their first term (odd chunks start at an
// odd k), after which the sign of step t is (-1)^t in every lane.
//
// The term prod_i f_i is kept as suffix products S_i = prod_{i' >= i} |f_i'| (S_m = 1) and
// sign words G_i = f_i xor G_{i+1} whose bit 31 is the parity of the negative f_i', i' >= i.
// Rows are sorted by the first Gray column that touches them, so a flip of column j changes
// only rows below hi[j]. Rows are recomputed in blocks with fixed bounds, fine where most
// flips end and coarse below them: block tops 2, 3, 4, 5, 6, 8, then every 4 rows. A flip of
// column j recomputes S and G in every block from the one holding row hi[j]-1 down to block
// 0 (rows of that top block above hi[j] are recomputed redundantly but exactly). Only S and
// G at block boundaries live across steps, which keeps the register footprint small. The
// top block of every column j < c is found once per item and packed, four bits per column,
// into one 64-bit scalar.
//
// The row values f_i are integers of magnitude below 2^24 (row sums are below 2^24), held as
// FP32, where every such integer and every sum of two of them that stays below 2^24 is exact:
// an update is one FMA with the signed delta, |f_i| is one conversion with the absolute-value
// source modifier, and the sign is bit 31 of the FP32 word.
//
// The deltas 2 b_ij of the Gray columns that flip inside the item (j < c) sit in LDS as a
// dense FP32 table D[j][row], one table per wave, written at the start of the item; a block's
// rows are read with one broadcast LDS load. All register arrays are indexed by constants.
constexpr int CMAX = 12;    // largest lane chunk exponent c (host clamps chunk_log2)

__host__ __device__ constexpr int blk_top(int b) { return b < 5 ? b + 2 : (b == 5 ? 8 : 8 + 4 * (b - 5)); }
__host__ __device__ constexpr int blk_lo(int b) { return b == 0 ? 0 : blk_top(b - 1); }

template <int MAXM>
struct Blocks {
    static constexpr int count() {
        int b = 0;
        while (blk_top(b) < MAXM) ++b;
        return b + 1;
    }
    static constexpr int N = count();   // blocks covering rows 0 .. MAXM-1
    static_assert(N <= 15, "four bits per packed block index");
};

template <int MAXM>
struct Tab {
    static constexpr int STRIDE = (blk_top(Blocks<MAXM>::N - 1) + 3) / 4 * 4;   // words per column
    static constexpr int WORDS = CMAX * STRIDE;                                // per wave
};

// Index of the block that holds row h-1 (h >= 1; h = 0 maps to block 0).
__device__ __forceinline__ uint32_t block_of(uint32_t h) {
    return h <= 6 ? (h <= 2 ? 0u : h - 2) : (h <= 8 ? 5u : 5u + (h - 5) / 4);
}

// Recompute block B (rows blk_lo(B) .. blk_top(B)-1, top row first) after a flip with the
// column's deltas dj (FP32, one per row) in direction dir.
#define HP_BLOCK(B)                                                                        \
    if ((B) < NB) {                                                                        \
        const int lo_ = blk_lo(B), w_ = blk_top(B) - blk_lo(B);                            \
        float dd_[4];                                                                      \
        if (w_ == 4) {                                                                     \
            const float4 v_ = *reinterpret_cast<const float4 *>(dj + lo_);                 \
            dd_[0] = v_.x;                                                                 \
            dd_[1] = v_.y;                                                                 \
            dd_[2] = v_.z;                                                                 \
            dd_[3] = v_.w;                                                                 \
        } else if (w_ == 2) {                                                              \
            const float2 v_ = *reinterpret_cast<const float2 *>(dj + lo_);                 \
            dd_[0] = v_.x;                                                                 \
            dd_[1] = v_.y;                                                                 \
        } else {                                                                           \
            dd_[0] = dj[lo_];                                                              \
        }                                                                                  \
        _Pragma("unroll") for (int r_ = 3; r_ >= 0; --r_) {                                \
            const int I_ = lo_ + r_;                                                       \
            if (r_ < w_ && I_ < MAXM) {                                                    \
                f[I_] = __builtin_fmaf(dd_[r_], dir, f[I_]);                               \
                G[I_] = G[I_ + 1] ^ __float_as_uint(f[I_]);                                \
                S[I_] = S[I_ + 1];                                                         \
                R::mul(S[I_], (uint32_t)fabsf(f[I_]));                                     \
            }                                                                              \
        }                                                                                  \
    }

// A flip: recompute the blocks from top block TOP down to block 0 with deltas DJ and
// direction DIR (one guard for the coarse blocks 5 and up, then one per fine block; plain
// ifs keep the control flow structured).
#define HP_FLIP(TOP, DJ, DIR)                                                              \
    {                                                                                      \
        const uint32_t top_ = (TOP);                                                       \
        const float *const dj = (DJ);                                                      \
        const float dir_ = (DIR);                                                          \
        const float dir = dir_;                                                            \
        const uint32_t top = top_;                                                         \
        if (top >= 5) {                                                                    \
            _Pragma("unroll") for (int B = NB - 1; B >= 5; --B) if ((int)top >= B) {       \
                HP_BLOCK(B)                                                                \
            }                                                                              \
        }                                                                                  \
        if (top >= 4) { HP_BLOCK(4) }                                                      \
        if (top >= 3) { HP_BLOCK(3) }                                                      \
        if (top >= 2) { HP_BLOCK(2) }                                                      \
        if (top >= 1) { HP_BLOCK(1) }                                                      \
        HP_BLOCK(0)                                                                        \
    }

// Row-value update of block B only (no product), for the rows below the pair boundary in
// the paired walk below.
#define HP_BLOCK_F(B)                                                                      \
    if ((B) < NB) {                                                                        \
        const int lo_ = blk_lo(B), w_ = blk_top(B) - blk_lo(B);                            \
        _Pragma("unroll") for (int r_ = 3; r_ >= 0; --r_) {                                \
            const int I_ = lo_ + r_;                                                       \
            if (r_ < w_ && I_ < MAXM) f[I_] = __builtin_fmaf(dj[I_], dir, f[I_]);          \
        }                                                                                  \
    }

// A flip in the paired walk: blocks V and up are recomputed in full, the blocks below the
// pair boundary (rows 0 .. V) only get their new row values.
#define HP_FLIP_P(TOP, DJ, DIR)                                                            \
    {                                                                                      \
        const uint32_t top_ = (TOP);                                                       \
        const float *const dj = (DJ);                                                      \
        const float dir_ = (DIR);                                                          \
        const float dir = dir_;                                                            \
        const uint32_t top = top_;                                                         \
        if (top >= 5) {                                                                    \
            _Pragma("unroll") for (int B = NB - 1; B >= 5; --B) if ((int)top >= B) {       \
                HP_BLOCK(B)                                                                \
            }                                                                              \
        }                                                                                  \
        if (top >= 4) { HP_BLOCK(4) }                                                      \
        if (top >= 3) { HP_BLOCK(3) }                                                      \
        if (top >= 2) { HP_BLOCK(2) }                                                      \
        if (V == 1) {                                                                      \
            if (top >= 1) { HP_BLOCK(1) }                                                  \
        } else {                                                                           \
            HP_BLOCK_F(1)                                                                  \
        }                                                                                  \
        HP_BLOCK_F(0)                                                                      \
    }

// A flip in the four-step walks (QB = 4 or 5, the block whose first row is the boundary row):
// blocks QB and up are recomputed in full, the blocks below (rows of A and B, whose values
// are held without columns 0 and 1) only get their new row values.
#define HP_FLIP_Q(TOP, DJ, DIR, QB)                                                        \
    {                                                                                      \
        const uint32_t top_ = (TOP);                                                       \
        const float *const dj = (DJ);                                                      \
        const float dir_ = (DIR);                                                          \
        const float dir = dir_;                                                            \
        const uint32_t top = top_;                                                         \
        if (top >= 5) {                                                                    \
            _Pragma("unroll") for (int B = NB - 1; B >= 5; --B) if ((int)top >= B) {       \
                HP_BLOCK(B)                                                                \
            }                                                                              \
        }                                                                                  \
        if ((QB) <= 4) { if (top >= 4) { HP_BLOCK(4) } } else { HP_BLOCK_F(4) }           \
        if ((QB) <= 3) { if (top >= 3) { HP_BLOCK(3) } } else { HP_BLOCK_F(3) }           \
        if ((QB) <= 2) { if (top >= 2) { HP_BLOCK(2) } } else { HP_BLOCK_F(2) }           \
        if ((QB) <= 1) { if (top >= 1) { HP_BLOCK(1) } } else { HP_BLOCK_F(1) }           \
        HP_BLOCK_F(0)                                                                      \
    }

// V = 0: the walk in step pairs below, for every job. V = 1, 2 (jobs whose column 0 reaches
// only the first b = V + 1 rows, lane chunks of at least 2 Gray indices): the paired walk.
// The two terms of a pair (t even, t + 1) differ only in Gray column 0, so rows 0 .. b-1 are
// held without it (g_i; column 0's deltas are d_i) and the pair is summed at once as
//   +-sign(G_b) * S_b * X,  X = prod_{i<b} (g_i + d_i) - prod_{i<b} g_i,
// with the plus sign when column 0 is set in the first term of the pair, and S_b, G_b the
// suffix product and sign word of the rows above. X is a small integer, exact in the ring's
// Small type; for b = 2 it is d_0 g_1 + d_1 g_0 + d_0 d_1. The other flips recompute S and G
// only from row b up and move g_0 .. g_{b-1}.
template <class R, int MAXM, int V0>
__device__ __forceinline__ void rnw_item(const JobDesc &jd, const uint32_t *__restrict__ data,
                                         uint64_t item, int lane, JobAcc *dst, float *tab) {
    static_assert(MAXM <= 40, "job orders up to 40");
    static_assert(V0 >= 0 && V0 <= 4, "walk variant");
    // V = 3, 4, the four-step walks, exist for the 64-bit ring only (the host gives them no
    // other jobs, and the other rings have no such kernels)
    static_assert(V0 < 3 || R::kFourStep, "four-step walks are mod 2^64 only");
    constexpr int V = V0;
    constexpr int STRIDE = Tab<MAXM>::STRIDE;
    constexpr int NB = Blocks<MAXM>::N;
    const int m = jd.m;
    const int c = jd.chunk_log2;
    const uint64_t nterms = 1ull << (m - 1);
    const uint64_t L = 1ull << c;
    const uint64_t z = item * WAVE + (uint64_t)lane;   // the lane's chunk
    const uint64_t k0 = z * L;
    const uint64_t kfirst = (z & 1) ? k0 + L - 1 : k0;   // the lane's first Gray index
    const uint32_t *w = data + (size_t)jd.data_off * HP_DATA_ALIGN;
    const uint32_t *cs = w + m;
    const uint32_t *hi = w + 2 * m;
    const uint32_t *ent = w + 3 * m;

    // delta table of the Gray columns 0..c-1 and their packed top blocks
    for (int q = lane; q < CMAX * STRIDE; q += WAVE) tab[q] = 0.0f;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint64_t tops = 0;
    for (int j = 0; j < c; ++j) {
        const uint32_t b = uni(cs[j]);
        const uint32_t n = uni(cs[j + 1]) - b;
        if ((uint32_t)lane < n) {
            const uint32_t pk = ent[b + lane];
            tab[j * STRIDE + (int)(pk & 0xff)] = (float)(int)(pk >> 8);
        }
        tops |= (uint64_t)block_of(uni(hi[j])) << (4 * j);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // f_i(gray(kfirst)) = base_i + 2 * sum over the set Gray bits. Bits 0..c-1 of
    // gray(kfirst) are zero, so only columns c .. m-2 can contribute; rows are selected by
    // comparison so that the row values stay in registers with constant indices.
    float f[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) f[i] = i < m ? (float)(int)uni(w[i]) : 1.0f;
    const uint64_t g0 = kfirst ^ (kfirst >> 1);
    for (int j = c; j < m - 1; ++j) {
        const bool bit = (g0 >> j) & 1;
        const uint32_t b = uni(cs[j]);
        const uint32_t e = uni(cs[j + 1]);
        for (uint32_t q = b; q < e; ++q) {
            const uint32_t pk = uni(ent[q]);
            const int row = (int)(pk & 0xff);
            const float d = bit ? (float)(int)(pk >> 8) : 0.0f;
#pragma unroll
            for (int i = 0; i < MAXM; ++i)
                if (row == i) f[i] += d;
        }
    }
    typename R::P S[MAXM + 1];
    uint32_t G[MAXM + 1];
    S[MAXM] = R::one();
    // the sign (-1)^kfirst of the lane's first term rides in the sign chain's seed; the sign
    // (-1)^t of step t relative to it is wave-uniform
    G[MAXM] = (uint32_t)(kfirst & 1) << 31;
#pragma unroll
    for (int i = MAXM - 1; i >= 0; --i) {
        S[i] = S[i + 1];
        G[i] = G[i + 1];
        if (i < m) {
            G[i] ^= __float_as_uint(f[i]);
            R::mul(S[i], (uint32_t)fabsf(f[i]));
        }
    }

    typename R::Acc acc = R::acc_zero();
    const uint32_t last = (uint32_t)L - 1u;
    const uint32_t top0 = (uint32_t)tops & 15u;
    if constexpr (V == 0) {
        // Steps come in pairs: an even term, the flip of column 0 (every other step; its top
        // block is fixed for the item), an odd term, then the flip of column j = ctz(t+1) >= 1.
        for (uint32_t t = 0;; ++t) {
            R::acc(acc, S[0], (uint32_t)((int)G[0] >> 31));   // even t: (-1)^t = +1
            if (t == last) break;
            {
                const float dir0 = __uint_as_float(0x3f800000u | ((((t + 1) >> 1) & 1u) << 31));
                HP_FLIP(top0, tab, dir0)
            }
            ++t;
            R::acc(acc, S[0], ~(uint32_t)((int)G[0] >> 31));   // odd t: (-1)^t = -1
            if (t == last) break;
            {
                const int j = __builtin_ctz(t + 1);
                const float dirj = __uint_as_float(0x3f800000u | ((((t + 1) >> (j + 1)) & 1u) << 31));
                HP_FLIP((uint32_t)(tops >> (4 * j)) & 15u, tab + j * STRIDE, dirj)
            }
        }
    } else if constexpr (V >= 3) {
        // Four-step walks (mod 2^64 jobs flagged by the host, lane chunks of at least 4 steps),
        // V = 3 with HA = 2, V = 4 with HA = 3: Gray column 0 touches exactly rows 0..HA-1 (A)
        // and column 1 only rows of HA..HB-1, HB = HA + 3 (B; a row of B that column 1 misses
        // is a factor of both B products and so of the sum); f holds rows 0..HB-1 with both
        // columns out. In the block of steps t..t+3 (t = 4q) every other column is fixed and
        // the four terms, with signs (-1)^q (+, -, +, -) in the reflected code's order, sum to
        // (-1)^q (A0 - A1)(B0 - B1) times the rows from HB up: A0, A1 the products of A
        // without and with column 0, B0, B1 those of B without and with column 1. One
        // multiply of the suffix S_HB per four terms, and the flips (columns 2 and up)
        // recompute the suffix products from row HB up only (HB is a block's first row: block
        // QB and up are recomputed in full, the blocks below get their new row values).
        constexpr int HA = V - 1;
        constexpr int HB = HA + 3;
        constexpr int QB = HA == 2 ? 4 : 5;
        // column 0's deltas on rows 0..HA-1 and column 1's on rows HA..HB-1 (wave-uniform)
        float dA[HA], dB[3];
#pragma unroll
        for (int i = 0; i < HA; ++i) dA[i] = __uint_as_float(uni(__float_as_uint(tab[i])));
#pragma unroll
        for (int i = 0; i < 3; ++i) dB[i] = __uint_as_float(uni(__float_as_uint(tab[STRIDE + HA + i])));
        // Block sum. The host gives these walks only jobs whose rows 0..HB-1 have row sums
        // below 2^7, so every value of those rows, with or without a column, is an integer
        // below 2^7 in magnitude: products of up to three are below 2^21 and A1 - A0, B1 - B0
        // below 2^22, all exact in FP32 (the last product and difference fused). The two
        // differences then go through the 24-bit multiplier (low and high halves, full rate)
        // into the 64-bit x = (A1 - A0)(B1 - B0) = (A0 - A1)(B0 - B1), and only the suffix
        // multiply is 64-bit.
#define HP_QUAD_BLOCK()                                                                    \
    {                                                                                      \
        float da;                                                                          \
        if constexpr (HA == 2) {                                                           \
            da = __builtin_fmaf(f[0] + dA[0], f[1] + dA[1], -(f[0] * f[1]));               \
        } else {                                                                           \
            const float a0 = f[0] * f[1] * f[2];                                           \
            da = __builtin_fmaf((f[0] + dA[0]) * (f[1] + dA[1]), f[2] + dA[2], -a0);       \
        }                                                                                  \
        const float b0 = f[HA] * f[HA + 1] * f[HA + 2];                                    \
        const float db = __builtin_fmaf((f[HA] + dB[0]) * (f[HA + 1] + dB[1]), f[HA + 2] + dB[2], -b0); \
        int64_t x = (int64_t)s24((int)da) * (int64_t)s24((int)db);                         \
        /* keep x one 24-bit product (the compiler would otherwise multiply S by each    */ \
        /* difference in turn, two 64 x 32-bit products)                                 */ \
        asm("" : "+v"(x));                                                                 \
        const uint32_t smask = 0u - ((t >> 2) & 1u);   /* all ones: minus (odd blocks) */  \
        R::acc(acc, R::pair_mul(S[HB], x), (uint32_t)((int)G[HB] >> 31) ^ smask);          \
    }
        // Blocks at t = 0, 4, .., L - 4 (L is a multiple of 4: the host gives this walk c >= 2).
        // Between blocks t and t + 4 column ctz(t + 4) >= 2 flips: column 2 after every other
        // block (its top block fixed for the item), a higher column after the rest.
        const uint32_t top2 = (uint32_t)(tops >> 8) & 15u;
        uint32_t t = 0;
        HP_QUAD_BLOCK()
        while ((uint64_t)t + 4 < L) {   // t is a multiple of 8 here
            {
                const float dir2 = __uint_as_float(0x3f800000u | ((((t + 4) >> 3) & 1u) << 31));
                HP_FLIP_Q(top2, tab + 2 * STRIDE, dir2, QB)
            }
            t += 4;
            HP_QUAD_BLOCK()
            if ((uint64_t)t + 4 >= L) break;
            {
                const int j = __builtin_ctz(t + 4);   // >= 3
                const float dirj = __uint_as_float(0x3f800000u | ((((t + 4) >> (j + 1)) & 1u) << 31));
                HP_FLIP_Q((uint32_t)(tops >> (4 * j)) & 15u, tab + j * STRIDE, dirj, QB)
            }
            t += 4;
            HP_QUAD_BLOCK()
        }
#undef HP_QUAD_BLOCK
    } else {
        constexpr int PB = V + 1;   // rows 0 .. PB-1 below the pair boundary
        using Sm = typename R::Small;
        // column 0's deltas d_i (wave-uniform) and, for PB = 2, d_0 d_1
        int dcol[PB];
#pragma unroll
        for (int i = 0; i < PB; ++i) dcol[i] = (int)__uint_as_float(uni(__float_as_uint(tab[i])));
        // (read back through the scalar unit so that the compiler keeps d_0 g_1 and d_1 g_0 as
        // two 32 x 32 -> 64-bit products instead of factoring d_0 (g_1 + d_1))
        const Sm k01 = (Sm)(int64_t)uni64((uint64_t)((int64_t)dcol[0] * dcol[1]));
        // Pair at t: column 0 is set in term t when bit 1 of t is (in every lane); the pair's
        // first term has the sign (-1)^kfirst of G's seed.
#define HP_PAIR()                                                                          \
    {                                                                                      \
        Sm x;                                                                              \
        if constexpr (PB == 2) {                                                           \
            x = k01 + (Sm)dcol[0] * (Sm)(int)f[1] + (Sm)dcol[1] * (Sm)(int)f[0];           \
        } else {                                                                           \
            /* X = d0 h1 h2 + g0 (d1 h2 + g1 d2), h = g + d: two 32 x 32 -> 64-bit       */ \
            /* products and two wider ones, in unsigned arithmetic (|X| < 2^74 wraps      */ \
            /* modulo 2^64 in the 64-bit ring, exactly what that ring needs)             */ \
            using Um = typename R::USmall;                                                 \
            const int g0_ = (int)f[0], g1_ = (int)f[1], g2_ = (int)f[2];                   \
            const int h2_ = g2_ + dcol[2];                                                 \
            Sm a_ = (Sm)(g1_ + dcol[1]) * (Sm)h2_;                                         \
            /* keep h1 h2 one 32 x 32 -> 64-bit product (the compiler would otherwise form */ \
            /* d0 h2 first and multiply 64 x 64 bits)                                    */ \
            if constexpr (sizeof(Sm) == 8) asm("" : "+v"(a_));                             \
            const Sm b_ = (Sm)dcol[1] * (Sm)h2_ + (Sm)g1_ * (Sm)dcol[2];                   \
            x = (Sm)((Um)(uint32_t)dcol[0] * (Um)a_ + (Um)(Sm)g0_ * (Um)b_);               \
        }                                                                                  \
        const uint32_t smask = ((t >> 1) & 1u) - 1u;   /* all ones: minus */               \
        R::acc(acc, R::pair_mul(S[PB], x), (uint32_t)((int)G[PB] >> 31) ^ smask);          \
    }
        // Flips between pairs: column j = ctz(t + 2) >= 1, direction from bit j + 1 of t + 2.
        uint32_t t = 0;
        HP_PAIR()
        while (t + 1 != last) {
            const int j = __builtin_ctz(t + 2);
            const float dirj = __uint_as_float(0x3f800000u | ((((t + 2) >> (j + 1)) & 1u) << 31));
            HP_FLIP_P((uint32_t)(tops >> (4 * j)) & 15u, tab + j * STRIDE, dirj)
            t += 2;
            HP_PAIR()
        }
#undef HP_PAIR
    }
    if (k0 >= nterms) acc = R::acc_zero();   // lanes past the end of a short job contribute nothing
    R::flush(acc, dst, lane);
}
#undef HP_FLIP_Q
#undef HP_FLIP_P
#undef HP_BLOCK_F
#undef HP_FLIP
#undef HP_BLOCK


// Persistent kernel: every wave repeatedly takes the next work item of the queue. The
// queue is the list of jobs in scheduling order; item_end[s] is the number of items of
// the first s+1 queued jobs (jobs own contiguous item ranges). Every queued job has
// order at most MAXM (the host queues jobs by order bucket). The two-row paired walk of the
// order-20 bucket (the default cut-off's jobs) is held to 64 VGPRs, 8 waves per SIMD: it needs
// 66 unconstrained, and the one value that then spills is stored and reloaded once per item,
// outside the Gray loop. (The same limit made the three-row walk slower.)
template <class R, int MAXM, int V>
__global__ __launch_bounds__(BLOCK, (MAXM == 20 && (V == 1 || V == 3) ? 8 : 1)) void rnw_persistent(const JobDesc *__restrict__ jobs,
                                                        const uint32_t *__restrict__ data,
                                                        const uint32_t *__restrict__ queue,
                                                        const uint64_t *__restrict__ item_end,
                                                        uint32_t nqueue, uint64_t total_items,
                                                        unsigned long long *head,
                                                        JobAcc *__restrict__ accs) {
    __shared__ __attribute__((aligned(16))) float tabs[(BLOCK / WAVE) * Tab<MAXM>::WORDS];
    const int lane = threadIdx.x & (WAVE - 1);
    float *tab = tabs + (threadIdx.x >> 6) * Tab<MAXM>::WORDS;
    for (;;) {
        // Every lane takes part in the claim (lane 0 adds 1, the others 0) so that no
        // lane-dependent branch surrounds it: the whole wave then reads lane 0's claim.
        // With the claim inside `if (lane == 0)`, the loop can be compiled as divergent and
        // lanes 1..63 never see a new claim.
        const unsigned long long got = atomicAdd(head, lane == 0 ? 1ull : 0ull);
        const uint64_t g = uni64(got);
        if (g >= total_items) break;
        // smallest s with item_end[s] > g
        uint32_t lo = 0, hi = nqueue - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (uni64(item_end[mid]) > g) hi = mid;
            else lo = mid + 1;
        }
        const uint64_t first = lo ? uni64(item_end[lo - 1]) : 0;
        const uint32_t job = uni(queue[lo]);
        const JobDesc jd = load_job(jobs, job);
        rnw_item<R, MAXM, V>(jd, data, g - first, lane, accs + job, tab);
    }
}

// The same queue walk that also adds the shader-clock cycles from taking an item to finishing
// it into cycles[job] (the per-job work times of the scheduling study). It is a kernel of its
// own: sharing one loop body with the untimed kernel changed that kernel's register
// allocation by one scalar register, enough to cost it one wave per SIMD.
template <class R, int MAXM, int V>
__global__ __launch_bounds__(BLOCK) void rnw_persistent_timed(const JobDesc *__restrict__ jobs,
                                                              const uint32_t *__restrict__ data,
                                                              const uint32_t *__restrict__ queue,
                                                              const uint64_t *__restrict__ item_end,
                                                              uint32_t nqueue, uint64_t total_items,
                                                              unsigned long long *head,
                                                              JobAcc *__restrict__ accs,
                                                              unsigned long long *__restrict__ cycles) {
    __shared__ __attribute__((aligned(16))) float tabs[(BLOCK / WAVE) * Tab<MAXM>::WORDS];
    const int lane = threadIdx.x & (WAVE - 1);
    float *tab = tabs + (threadIdx.x >> 6) * Tab<MAXM>::WORDS;
    for (;;) {
        const unsigned long long got = atomicAdd(head, lane == 0 ? 1ull : 0ull);
        const uint64_t g = uni64(got);
        if (g >= total_items) break;
        uint32_t lo = 0, hi = nqueue - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (uni64(item_end[mid]) > g) hi = mid;
            else lo = mid + 1;
        }
        const uint64_t first = lo ? uni64(item_end[lo - 1]) : 0;
        const uint32_t job = uni(queue[lo]);
        const JobDesc jd = load_job(jobs, job);
        const uint64_t t0 = (uint64_t)clock64();
        rnw_item<R, MAXM, V>(jd, data, g - first, lane, accs + job, tab);
        const unsigned long long dt = (unsigned long long)((uint64_t)clock64() - t0);
        atomicAdd(cycles + job, lane == 0 ? dt : 0ull);
    }
}

// One launch per job (the plain comparator): wave w of the grid evaluates item w.
template <class R, int MAXM, int V>
__global__ __launch_bounds__(BLOCK) void rnw_single(const JobDesc *__restrict__ jobs,
                                                    const uint32_t *__restrict__ data,
                                                    uint32_t job, uint64_t nitems,
                                                    JobAcc *__restrict__ accs) {
    __shared__ __attribute__((aligned(16))) float tabs[(BLOCK / WAVE) * Tab<MAXM>::WORDS];
    const int lane = threadIdx.x & (WAVE - 1);
    float *tab = tabs + (threadIdx.x >> 6) * Tab<MAXM>::WORDS;
    const uint64_t w = (uint64_t)blockIdx.x * (BLOCK / WAVE) + (threadIdx.x >> 6);
    if (w >= nitems) return;
    const JobDesc jd = load_job(jobs, job);
    rnw_item<R, MAXM, V>(jd, data, w, lane, accs + job, tab);
}

#endif  // HP_PART >= 1

#if HP_PART == 0
// ------------------------------------------------------------------------ KKLLL estimate
// Counter-based SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output k of the stream
// seeded with s is mix(s + (k+1) * golden), golden = 0x9E3779B97F4A7C15.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Cube-root exponent of entry (i, j) of trial t of job w: counter (w<<36)|(t<<12)|(i<<6)|j,
// exponent floor(3 * (x >> 32) / 2^32).
__device__ __forceinline__ uint32_t kkl_u_counter(uint64_t seed, uint64_t k) {
    const uint64_t x = splitmix64(seed, k);
    return (uint32_t)(((x >> 32) * 3ull) >> 32);
}

// KKLLL on one job per block (4 waves). A wave holds 64 / GROUP trials at once, one per
// group of GROUP lanes (GROUP >= m); lane r of a group holds row r of that trial's B in
// registers (complex FP32, columns in job order). The matrix is written into LDS by all
// lanes (one random draw per nonzero), then each lane loads its row. Gaussian elimination
// with partial pivoting: the pivot row is the unused row with the largest |B_rk|, found by a
// butterfly inside the group and broadcast with lane permutes; log|det B| is the sum of
// log|pivot|. Trials accumulate log-sum-exp pairs; the key is log(mean |det B|^2).
// Maximum of a 32-bit key over aligned groups of GROUP lanes (16, 32 or 64): DPP steps
// inside rows of 16 lanes (quad swaps, half-row and row mirrors), then the row swaps of
// gfx950 (v_permlane16_swap: neighbouring 16-lane rows; v_permlane32_swap: the two halves),
// whose two results hold each lane's value and its partner's, so their maximum is the pair's.
template <int GROUP>
__device__ __forceinline__ uint32_t group_max(uint32_t x) {
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false));    // lane ^ 1
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false));    // lane ^ 2
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false));   // 7 - lane in 8
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false));   // 15 - lane in 16
    if (GROUP >= 32) {   // lane ^ 16
        const auto s = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        x = max((uint32_t)s[0], (uint32_t)s[1]);
    }
    if (GROUP >= 64) {   // lane ^ 32
        const auto s = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        x = max((uint32_t)s[0], (uint32_t)s[1]);
    }
    return x;
}

template <int MAXM, int GROUP>
struct KklShape {
    static_assert(MAXM <= GROUP && (GROUP == 16 || GROUP == 32 || GROUP == 64), "group size");
    static constexpr int TPW = WAVE / GROUP;              // trials per wave pass
    static constexpr int LD = (MAXM + 3) / 4 * 4;         // row length in bytes (entry codes)
    static constexpr int WAVE_BYTES = TPW * MAXM * LD;    // entry codes per wave
};

// Entry code of a staged matrix: 0 for a structural zero, 1 + u for omega^u.
__device__ __forceinline__ void kkl_decode(uint32_t code, float &re, float &im) {
    constexpr float kS = 0.86602540378443864676f;   // sin(2 pi / 3)
    re = code == 1 ? 1.0f : (code != 0 ? -0.5f : 0.0f);
    im = code == 2 ? kS : (code == 3 ? -kS : 0.0f);
}

// Gaussian elimination with partial pivoting of one trial's B, held one row per lane of a
// group (z: this lane's row, real and imaginary parts interleaved), returning
// log2 |det B|^2 (the sum of log2 |pivot|^2). `singular` is set when a pivot is zero (and must
// come in set for a group without a trial). At every step the pivot lane writes its row, from
// the aligned column pair holding the pivot column on, into the group's LDS row `prow` with
// 16-byte stores, and the group reads it back with 16-byte broadcast loads (two columns per
// load: half the LDS cycles of moving the values one 32-bit lane permute at a time).
template <int MAXM, int GROUP>
__device__ __forceinline__ float kkl_eliminate(float (&z)[2 * MAXM], int m, int r, bool &singular,
                                               float *prow) {
    static_assert(MAXM % 2 == 0, "rows are written in column pairs");
    bool used = r >= m;
    float l2 = 0.0f;
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
        if (k < m) {
            // pivot: the unused row with the largest |B_rk|^2, as a packed key (the squared
            // magnitude's FP32 bits with the low 6 bits replaced by 63 - row, so that equal
            // magnitudes prefer the lower row) maximised inside the group
            const float mag = __builtin_fmaf(z[2 * k], z[2 * k], z[2 * k + 1] * z[2 * k + 1]);
            const uint32_t key = used ? 0u : ((__float_as_uint(mag) & ~63u) | (uint32_t)(63 - r));
            const int idx = 63 - (int)(group_max<GROUP>(key) & 63u);
            const int k0 = k & ~1;   // a constant once the loop is unrolled
            if (r == idx) {
#pragma unroll
                for (int c = k0; c < MAXM; c += 2)
                    if (c < m)
                        *reinterpret_cast<float4 *>(prow + 2 * c) =
                            make_float4(z[2 * c], z[2 * c + 1], z[2 * c + 2], z[2 * c + 3]);
                used = true;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const float4 q0 = *reinterpret_cast<const float4 *>(prow + 2 * k0);
            const float pr = (k & 1) ? q0.z : q0.x, pi = (k & 1) ? q0.w : q0.y;
            const float pmag = __builtin_fmaf(pr, pr, pi * pi);
            const bool ok = !singular && pmag > 0.0f;
            singular = !ok;
            const float pm = ok ? pmag : 1.0f;
            // hardware log2 and reciprocal (about 1 ulp): ample for a key that only orders
            // the queue
            l2 += __builtin_amdgcn_logf(pm);
            const float inv = __builtin_amdgcn_rcpf(pm);
            // factor = B_rk / pivot (zero for used rows and failed groups)
            const float ir = pr * inv, ii = -pi * inv;
            const bool upd = ok && !used;
            const float fr = upd ? __builtin_fmaf(z[2 * k], ir, -z[2 * k + 1] * ii) : 0.0f;
            const float fi = upd ? __builtin_fmaf(z[2 * k], ii, z[2 * k + 1] * ir) : 0.0f;
            // B_rc -= f * B_pc for c > k, as two fused multiply-adds per part
#define HP_KKL_UPD(C, CR, CI)                                                                  \
    z[2 * (C)] = __builtin_fmaf(-fr, (CR), __builtin_fmaf(fi, (CI), z[2 * (C)]));              \
    z[2 * (C) + 1] = __builtin_fmaf(-fr, (CI), __builtin_fmaf(-fi, (CR), z[2 * (C) + 1]));
            // (a pair's second column may lie past m: its entries are zero in every row and
            // stay zero, and no later step reads it)
            if (k == k0) { HP_KKL_UPD(k + 1, q0.z, q0.w) }
#pragma unroll
            for (int c = k0 + 2; c < MAXM; c += 2) {
                if (c < m) {
                    const float4 q = *reinterpret_cast<const float4 *>(prow + 2 * c);
                    HP_KKL_UPD(c, q.x, q.y)
                    HP_KKL_UPD(c + 1, q.z, q.w)
                }
            }
#undef HP_KKL_UPD
            // the next pivot lane may overwrite the row only after every lane has read it
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    return l2;
}

template <int MAXM, int GROUP>
__global__ __launch_bounds__(BLOCK, (MAXM <= 24 ? 6 : 3)) void kkl_estimate(const JobDesc *__restrict__ jobs,
                                                      const uint32_t *__restrict__ data,
                                                      const uint32_t *__restrict__ list,
                                                      uint32_t nlist, int trials, uint64_t seed,
                                                      float *__restrict__ keys) {
    using Sh = KklShape<MAXM, GROUP>;
    __shared__ __attribute__((aligned(16))) uint8_t mats[(BLOCK / WAVE) * Sh::WAVE_BYTES];
    __shared__ uint32_t ekey[MAXM * MAXM];   // Gray entries (at most m(m-1)) + m fixed slots
    __shared__ uint16_t epos[MAXM * MAXM];
    __shared__ float red[2 * (BLOCK / WAVE)];
    __shared__ __attribute__((aligned(16))) float prows[(BLOCK / WAVE) * Sh::TPW * 2 * MAXM];
    if (blockIdx.x >= nlist) return;
    const uint32_t jobid = uni(list[blockIdx.x]);
    const JobDesc jd = load_job(jobs, jobid);
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x >> 6;
    const int grp = lane / GROUP;             // trial slot inside the wave
    const int r = lane % GROUP;               // row held by this lane
    const int m = jd.m;
    const int nnz = (int)jd.nnz;
    const uint32_t *w = data + (size_t)jd.data_off * HP_DATA_ALIGN;
    const uint32_t *cs = w + m;
    const uint32_t *ent = w + 3 * m;
    const uint32_t *cmap = w + 3 * m + jd.nnz;
    const uint32_t *rmap = cmap + m;
    uint8_t *wm = mats + wave * Sh::WAVE_BYTES;

    // The job's nonzeros once per block: for entry e, the counter bits (original row << 6 |
    // original column, of the untransposed sub-matrix) of its random draw and its byte
    // position in a staged matrix. Gray entries first (thread j < m-1 takes Gray column j's
    // entries, so the loads of all columns are in flight at once), then one slot per row for
    // the fixed column: b_i,fixed = base_i + the row's Gray entries, summed by LDS atomics into
    // fixv (a zero entry gets no draw).
    __shared__ int fixv[MAXM];
    const int tid = threadIdx.x;
    const bool tr = (jd.flags & HP_FLAG_TRANSPOSED) != 0;   // draws follow the untransposed job
    if (tid < m) fixv[tid] = (int)w[tid];
    __syncthreads();
    if (tid < m - 1) {
        const uint32_t b = cs[tid], e = cs[tid + 1];
        const uint32_t ccol = cmap[tid];
        for (uint32_t q = b; q < e; ++q) {
            const uint32_t pk = ent[q];
            const int row = (int)(pk & 0xff);
            atomicAdd(&fixv[row], (int)(pk >> 9));
            const uint32_t rr = rmap[row];
            ekey[q] = tr ? ((ccol << 6) | rr) : ((rr << 6) | ccol);
            epos[q] = (uint16_t)(row * Sh::LD + tid);
        }
    }
    __syncthreads();
    if (tid < m) {
        const bool nz = fixv[tid] != 0;
        ekey[nnz + tid] = !nz ? ~0u : tr ? ((cmap[m - 1] << 6) | rmap[tid]) : ((rmap[tid] << 6) | cmap[m - 1]);
        epos[nnz + tid] = (uint16_t)(tid * Sh::LD + (m - 1));
    }
    __syncthreads();
    const int nent = nnz + m;

    float run_max = -INFINITY, run_sum = 0.0f;   // per lane; identical within a group
    for (int t0 = wave * Sh::TPW; t0 < trials; t0 += (BLOCK / WAVE) * Sh::TPW) {
        const int t = t0 + grp;                      // this group's trial
        const bool live = t < trials;
        // zero the wave's matrices, then write the nonzeros (all lanes share the work)
        for (int q = lane; q < Sh::WAVE_BYTES / 4; q += WAVE) reinterpret_cast<uint32_t *>(wm)[q] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int g = 0; g < Sh::TPW; ++g) {
            const int tg = t0 + g;
            if (tg >= trials) break;
            uint8_t *mg = wm + g * MAXM * Sh::LD;
            const uint64_t cbase = ((uint64_t)jobid << 36) | ((uint64_t)tg << 12);
            for (int e = lane; e < nent; e += WAVE) {
                const uint32_t key = ekey[e];
                if (key != ~0u) mg[epos[e]] = (uint8_t)(1 + kkl_u_counter(seed, cbase | key));
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float z[2 * MAXM];   // this lane's row: real and imaginary parts interleaved
        const uint32_t *myrow =
            reinterpret_cast<const uint32_t *>(wm + grp * MAXM * Sh::LD + (r < MAXM ? r : 0) * Sh::LD);
#pragma unroll
        for (int q = 0; q < Sh::LD / 4; ++q) {
            const uint32_t word = r < m ? myrow[q] : 0u;
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (4 * q + b < MAXM) kkl_decode((word >> (8 * b)) & 0xffu, z[2 * (4 * q + b)], z[2 * (4 * q + b) + 1]);
        }
        bool singular = !live;
        // log2 |det B|^2
        const float l2 = kkl_eliminate<MAXM, GROUP>(z, m, r, singular, prows + (wave * Sh::TPW + grp) * 2 * MAXM);
        if (!singular) {
            const float l = l2 * 0.69314718055994531f;   // log |det B|^2
            if (l > run_max) {
                run_sum = run_sum * __expf(run_max - l) + 1.0f;
                run_max = l;
            } else {
                run_sum += __expf(l - run_max);
            }
        }
    }
    // combine the (max, sum) pairs of all groups of all waves (one per group's first lane):
    // log-sum-exp butterflies inside the wave, then the four waves' pairs through LDS
    float mx = r == 0 ? run_max : -INFINITY;
    float sm = r == 0 ? run_sum : 0.0f;
#pragma unroll
    for (int sft = 32; sft >= 1; sft >>= 1) {
        const float om = __shfl_xor(mx, sft, WAVE);
        const float os = __shfl_xor(sm, sft, WAVE);
        const float nm = fmaxf(mx, om);
        sm = (mx > -INFINITY ? sm * __expf(mx - nm) : 0.0f) + (om > -INFINITY ? os * __expf(om - nm) : 0.0f);
        mx = nm;
    }
    if (lane == 0) {
        red[2 * wave] = mx;
        red[2 * wave + 1] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float m4 = -INFINITY;
        for (int v = 0; v < BLOCK / WAVE; ++v) m4 = fmaxf(m4, red[2 * v]);
        float sum = 0.0f;
        if (m4 > -INFINITY)
            for (int v = 0; v < BLOCK / WAVE; ++v)
                if (red[2 * v] > -INFINITY) sum += red[2 * v + 1] * __expf(red[2 * v] - m4);
        keys[jobid] = (m4 > -INFINITY && sum > 0.0f) ? m4 + __logf(sum) - __logf((float)trials)
                                                     : -INFINITY;
    }
}

// Step 4 of Algorithm PH on the device: every job's ring value V is turned into its
// permanent and added into its problem's accumulator (a normalised accumulator already holds
// the permanent).
//   mod 2^64 / 2^128: per = (-1)^(m-1) V / 2^(m-1); V must be divisible by 2^(m-1) with a
//   non-negative quotient (else the problem's error flag is set); the 32-bit limbs of per are
//   added into lim[0..3].
//   residues: per mod p_k = (-1)^(m-1) (2^-1)^(m-1) V mod p_k, added as 32-bit halves into
//   res[2k], res[2k+1]; the host reduces the sums and applies the CRT.
template <uint64_t C>
__device__ __forceinline__ uint64_t res_normalise(uint64_t lo_sum, uint64_t hi_sum, int m) {
    constexpr uint64_t P = (1ull << 61) - C;
    constexpr uint64_t INV2 = (P + 1) / 2;
    uint64_t v = mod61<C>((unsigned __int128)lo_sum + ((unsigned __int128)hi_sum << 32));
    for (int e = 0; e < m - 1; ++e) v = mulmod_full<C>(v, INV2);
    if (((m - 1) & 1) && v) v = P - v;
    return v;
}

__global__ void recombine(const JobDesc *__restrict__ jobs, const JobAcc *__restrict__ accs,
                          uint32_t njobs, ProbAcc *__restrict__ probs) {
    // contributions of this lane's job to its problem: lim[0..3] (32-bit limbs of per(B_w))
    // and res[0..5] (32-bit halves of the three residues of per(B_w))
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (WAVE - 1);
    uint64_t v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t problem = 0;
    bool bad = false;
    if (k < njobs) {
        const JobDesc d = jobs[k];
        const JobAcc a = accs[k];
        problem = d.problem;
        const int sh = d.m - 1;
        if (a.flag == HP_ACC_NORMALISED) {   // per(B) itself (device continuation of H_per)
            const unsigned __int128 per = (unsigned __int128)a.l[0] + ((unsigned __int128)a.l[1] << 32) +
                                          ((unsigned __int128)a.l[2] << 64) + ((unsigned __int128)a.l[3] << 96);
            v[0] = (uint32_t)per;
            v[1] = (uint32_t)(per >> 32);
            v[2] = (uint32_t)(per >> 64);
            v[3] = (uint32_t)(per >> 96);
        } else if (d.arith == HP_RES) {
            const uint64_t r0 = res_normalise<HP_C0>(a.l[0], a.l[1], d.m);
            const uint64_t r1 = res_normalise<HP_C1>(a.l[2], a.l[3], d.m);
            const uint64_t r2 = res_normalise<HP_C2>(a.l[4], a.l[5], d.m);
            v[4] = r0 & 0xffffffffull;
            v[5] = r0 >> 32;
            v[6] = r1 & 0xffffffffull;
            v[7] = r1 >> 32;
            v[8] = r2 & 0xffffffffull;
            v[9] = r2 >> 32;
        } else {
            unsigned __int128 V;
            if (d.arith == HP_W64) {
                const __int128 sv = (int64_t)a.l[0];
                V = (unsigned __int128)sv;
            } else {
                V = (unsigned __int128)a.l[0] + ((unsigned __int128)a.l[1] << 32) +
                    ((unsigned __int128)a.l[2] << 64) + ((unsigned __int128)a.l[3] << 96);
            }
            if (sh & 1) V = (unsigned __int128)0 - V;
            const bool neg = (V >> 127) != 0;
            const bool divisible = sh == 0 || (V & (((unsigned __int128)1 << sh) - 1)) == 0;
            if (neg || !divisible) {
                bad = true;
            } else {
                const unsigned __int128 per = V >> sh;
                v[0] = (uint32_t)per;
                v[1] = (uint32_t)(per >> 32);
                v[2] = (uint32_t)(per >> 64);
                v[3] = (uint32_t)(per >> 96);
            }
        }
    }
    if (bad) atomicOr(&probs[problem].err, 1u);
    // jobs in natural order are grouped by problem: when the whole wave holds one problem
    // (lanes past the end hold zeros), sum in the wave and add once per slot
    const uint32_t p0 = uni(problem);
    const bool same = k >= njobs || problem == p0;
    if (__ballot(!same) == 0) {
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            const uint64_t t = wave_sum64(v[q]);
            if (lane == 0 && t) {
                if (q < 4) atomicAdd(&probs[p0].lim[q], (unsigned long long)t);
                else atomicAdd(&probs[p0].res[q - 4], (unsigned long long)t);
            }
        }
    } else if (k < njobs) {
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            if (!v[q]) continue;
            if (q < 4) atomicAdd(&probs[problem].lim[q], (unsigned long long)v[q]);
            else atomicAdd(&probs[problem].res[q - 4], (unsigned long long)v[q]);
        }
    }
}

__global__ void fill_u64(unsigned long long *p, uint64_t n, unsigned long long v) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

#endif  // HP_PART == 0

}  // namespace

// ------------------------------------------------------------------------ launchers
namespace hp {

#if HP_PART == 0

int bucket_of(int m) { return m <= 16 ? 0 : (m <= 20 ? 1 : (m <= 24 ? 2 : (m <= 32 ? 3 : 4))); }

int est_bucket_of(int m) { return m <= 16 ? 0 : (m <= 20 ? 1 : (m <= 24 ? 2 : (m <= 32 ? 3 : 4))); }

int walk_variant(const JobDesc &d, int chunk_log2) {
    if (chunk_log2 < 1) return 0;
    if ((d.flags & HP_FLAG_QUAD) && d.arith == HP_W64 && chunk_log2 >= 2)
        return (d.flags & HP_FLAG_COL0_TWO_ROWS) ? 6 : 7;   // the four-step walks
    return (d.flags & HP_FLAG_COL0_TWO_ROWS) ? 1 : (d.flags & HP_FLAG_COL0_THREE_ROWS) ? 2 : 0;
}

hipError_t launch_recombine(const JobDesc *jobs, const JobAcc *accs, uint32_t njobs,
                            ProbAcc *probs, hipStream_t s) {
    if (njobs == 0) return hipSuccess;
    hipLaunchKernelGGL(recombine, dim3((njobs + 255) / 256), dim3(256), 0, s, jobs, accs, njobs, probs);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v,
                           hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(fill_u64, dim3((uint32_t)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_estimate(int bucket, const JobDesc *jobs, const uint32_t *data,
                           const uint32_t *list, uint32_t nlist, int trials, uint64_t seed,
                           float *keys, hipStream_t s) {
    if (nlist == 0) return hipSuccess;
    switch (bucket) {
        case 0: hipLaunchKernelGGL((kkl_estimate<16, 16>), dim3(nlist), dim3(BLOCK), 0, s, jobs, data, list, nlist, trials, seed, keys); break;
        case 1: hipLaunchKernelGGL((kkl_estimate<20, 32>), dim3(nlist), dim3(BLOCK), 0, s, jobs, data, list, nlist, trials, seed, keys); break;
        case 2: hipLaunchKernelGGL((kkl_estimate<24, 32>), dim3(nlist), dim3(BLOCK), 0, s, jobs, data, list, nlist, trials, seed, keys); break;
        case 3: hipLaunchKernelGGL((kkl_estimate<32, 32>), dim3(nlist), dim3(BLOCK), 0, s, jobs, data, list, nlist, trials, seed, keys); break;
        default: hipLaunchKernelGGL((kkl_estimate<HP_MAX_M, 64>), dim3(nlist), dim3(BLOCK), 0, s, jobs, data, list, nlist, trials, seed, keys);
    }
    return hipGetLastError();
}
#endif  // HP_PART == 0

#if HP_PART >= 1
// HP_V6, HP_V7: the kernels of launch variants 6 and 7 (the four-step walks, which only the
// 64-bit ring has; the host gives the other rings no such jobs)
#if HP_PART == 1
#define RING_T RingW64
#define RING_SUFFIX w64
#define HP_V6 3
#define HP_V7 4
#elif HP_PART == 2
#define RING_T RingW128
#define RING_SUFFIX w128
#define HP_V6 1
#define HP_V7 2
#else
#define RING_T RingRes
#define RING_SUFFIX res
#define HP_V6 1
#define HP_V7 2
#endif
#define CAT2(a, b) a##_##b
#define CAT(a, b) CAT2(a, b)

// Kernel of an order bucket and walk variant.
#define HP_FN(K, MAXM)                                                                     \
    (variant == 1   ? (const void *)K<RING_T, MAXM, 1>                                     \
     : variant == 2 ? (const void *)K<RING_T, MAXM, 2>                                     \
     : variant == 6 ? (const void *)K<RING_T, MAXM, HP_V6>                                 \
     : variant == 7 ? (const void *)K<RING_T, MAXM, HP_V7>                                 \
                    : (const void *)K<RING_T, MAXM, 0>)
static const void *persistent_fn(int bucket, int variant, bool timed) {
    if (!timed) {
        switch (bucket) {
            case 0: return HP_FN(rnw_persistent, 16);
            case 1: return HP_FN(rnw_persistent, 20);
            case 2: return HP_FN(rnw_persistent, 24);
            case 3: return HP_FN(rnw_persistent, 32);
            default: return HP_FN(rnw_persistent, HP_MAX_M);
        }
    }
    switch (bucket) {
        case 0: return HP_FN(rnw_persistent_timed, 16);
        case 1: return HP_FN(rnw_persistent_timed, 20);
        case 2: return HP_FN(rnw_persistent_timed, 24);
        case 3: return HP_FN(rnw_persistent_timed, 32);
        default: return HP_FN(rnw_persistent_timed, HP_MAX_M);
    }
}
static const void *single_fn(int bucket, int variant) {
    switch (bucket) {
        case 0: return HP_FN(rnw_single, 16);
        case 1: return HP_FN(rnw_single, 20);
        case 2: return HP_FN(rnw_single, 24);
        case 3: return HP_FN(rnw_single, 32);
        default: return HP_FN(rnw_single, HP_MAX_M);
    }
}
#undef HP_FN

hipError_t CAT(persistent_grid, RING_SUFFIX)(int bucket, int variant, int *grid) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_fn(bucket, variant, false), BLOCK, 0);
    if (e != hipSuccess) return e;
    *grid = cus * (per_cu > 0 ? per_cu : 1);
    return hipSuccess;
}

hipError_t CAT(launch_rnw_persistent, RING_SUFFIX)(int bucket, int variant, const JobDesc *jobs,
                                                    const uint32_t *data, const uint32_t *queue,
                                                    const uint64_t *item_end, uint32_t nqueue,
                                                    uint64_t total_items, unsigned long long *head,
                                                    JobAcc *accs, unsigned long long *cycles, int grid,
                                                    hipStream_t s) {
    void *args[] = {(void *)&jobs,   (void *)&data,        (void *)&queue, (void *)&item_end,
                    (void *)&nqueue, (void *)&total_items, (void *)&head,  (void *)&accs,
                    (void *)&cycles};   // the untimed kernel takes the first eight
    hipError_t e = hipLaunchKernel(persistent_fn(bucket, variant, cycles != nullptr), dim3(grid),
                                   dim3(BLOCK), args, 0, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t CAT(launch_rnw_single, RING_SUFFIX)(int bucket, int variant, const JobDesc *jobs,
                                                const uint32_t *data, uint32_t job, uint64_t nitems,
                                                JobAcc *accs, hipStream_t s) {
    const uint64_t blocks = (nitems + (BLOCK / WAVE) - 1) / (BLOCK / WAVE);
    void *args[] = {(void *)&jobs, (void *)&data, (void *)&job, (void *)&nitems, (void *)&accs};
    hipError_t e = hipLaunchKernel(single_fn(bucket, variant), dim3((uint32_t)blocks), dim3(BLOCK), args, 0, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}
#endif  // HP_PART >= 1

#if HP_PART == 0
hipError_t persistent_grid(int ring, int bucket, int variant, int *grid) {
    switch (ring) {
        case HP_W64: return persistent_grid_w64(bucket, variant, grid);
        case HP_W128: return persistent_grid_w128(bucket, variant, grid);
        default: return persistent_grid_res(bucket, variant, grid);
    }
}

hipError_t launch_rnw_persistent(int ring, int bucket, int variant, const JobDesc *jobs,
                                 const uint32_t *data, const uint32_t *queue,
                                 const uint64_t *item_end, uint32_t nqueue, uint64_t total_items,
                                 unsigned long long *head, JobAcc *accs,
                                 unsigned long long *cycles, int grid_override, hipStream_t s) {
    if (nqueue == 0 || total_items == 0) return hipSuccess;
    int grid = 0;
    hipError_t e = persistent_grid(ring, bucket, variant, &grid);
    if (e != hipSuccess) return e;
    if (grid_override > 0) grid = grid_override;
    const uint64_t max_blocks = (total_items + (BLOCK / WAVE) - 1) / (BLOCK / WAVE);
    if ((uint64_t)grid > max_blocks) grid = (int)max_blocks;
    switch (ring) {
        case HP_W64: return launch_rnw_persistent_w64(bucket, variant, jobs, data, queue, item_end, nqueue, total_items, head, accs, cycles, grid, s);
        case HP_W128: return launch_rnw_persistent_w128(bucket, variant, jobs, data, queue, item_end, nqueue, total_items, head, accs, cycles, grid, s);
        default: return launch_rnw_persistent_res(bucket, variant, jobs, data, queue, item_end, nqueue, total_items, head, accs, cycles, grid, s);
    }
}

hipError_t launch_rnw_single(int ring, int bucket, int variant, const JobDesc *jobs,
                             const uint32_t *data, uint32_t job, uint64_t nitems, JobAcc *accs,
                             hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    switch (ring) {
        case HP_W64: return launch_rnw_single_w64(bucket, variant, jobs, data, job, nitems, accs, s);
        case HP_W128: return launch_rnw_single_w128(bucket, variant, jobs, data, job, nitems, accs, s);
        default: return launch_rnw_single_res(bucket, variant, jobs, data, job, nitems, accs, s);
    }
}
#endif  // HP_PART == 0

}  // namespace hp
