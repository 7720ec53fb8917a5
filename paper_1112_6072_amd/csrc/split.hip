// Device continuation of Algorithm H_per (Section 2.1) below the host's cut-off, R-NW on the
// leaves it reaches, and their sum per job (Step 4 of Algorithm PH, inside one job).
//
// One wave takes one job (a sub-matrix B of order m <= HP_SPLIT_MAX_M, mod-2^64 arithmetic)
// from a queue and rebuilds it densely in its LDS region. It walks the H_per expansion tree
// of B depth first. At a node of order o, s is the smallest number of nonzeros in a row or a
// column (ties: rows first, then the lowest index). s = 0 drops the node (per = 0); a node with
// o <= t (the target order), o <= 2 or s >= s_leaf is a leaf; otherwise expansion (2) along
// that line gives ceil(s/2) <= 2 children of order o - 1: consecutive nonzeros of the line are
// paired and each pair's two columns (rows, for a column line) merged with crossed weights,
// an odd last nonzero paired at weight 0 with the lowest zero of the line. This is the rule of
// the host expansion. The nodes on the current path all have different orders, so each order
// has one LDS slot: the node of order o and its control state (line, pairs, next child) live
// at slot o. A split whose children would hold an entry >= 2^22 or a row sum >= 2^24 is not
// made: the node becomes a leaf (the bounds the host keeps for every job).
//
// A leaf of order p is evaluated by the whole wave with the doubled Nijenhuis-Wilf form of
// Ryser's formula (fixed column p - 1, Gray columns 0..p-2):
//     V = sum_k (-1)^k prod_i f_i(gray(k)) = (-1)^(p-1) 2^(p-1) per(leaf).
// Lane z walks the 2^(p-7) Gray indices of chunk z, odd chunks backwards. Then at step s every
// lane flips Gray column ctz(s) and adds it exactly when bit ctz(s) + 1 of s is clear (both
// hold in either direction of the reflected code), no lane's start subset holds a column below
// p - 7, and the term of step s has the sign (-1)^(s + z). Rows beyond p are padded with f = 1.
// Leaves are summed in the scale of the job,
//     (-1)^(m-1) 2^(m-1) per(B) = sum_leaves (-1)^(m-p) 2^(m-p) V_leaf   (mod 2^64),
// which is the value the per-item R-NW kernels leave in a job's accumulator, so the 2-adic
// check and the recombination of the jobs are shared with them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hperm_internal.h"
#include "kernels.h"

namespace hp {
namespace {

constexpr int SW = 64;                   // one wave per block
constexpr int SMAX = HP_SPLIT_MAX_M;     // largest job order
constexpr int DSTRIDE = 20;              // words per Gray column in a leaf's delta table
constexpr int CTL = 12;                  // control words per order

// LDS words of the node slots of orders o + 1 .. SMAX (the slot of order o starts there).
__host__ __device__ constexpr int slot_off(int o) {
    return (SMAX * (SMAX + 1) * (2 * SMAX + 1) - o * (o + 1) * (2 * o + 1)) / 6;
}
__host__ __device__ constexpr int align4(int w) { return (w + 3) & ~3; }
// Per-wave region for target order t: slots of orders t..SMAX, the leaf's delta table and
// base values, and the control words.
__host__ __device__ constexpr int region_words(int t) {
    return align4(slot_off(t - 1)) + SMAX * DSTRIDE + SMAX + (SMAX + 1) * CTL;
}
static_assert(align4(SMAX * DSTRIDE + SMAX) == SMAX * DSTRIDE + SMAX, "16-byte alignment of the tables");

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

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    for (int o = 32; o; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
    for (int o = 32; o; o >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, o);
    return v;
}

// floor(e / d) for e < 1024, 1 <= d <= 32 (multiply by the rounded-up reciprocal: exact here).
__device__ __forceinline__ uint32_t div_small(uint32_t e, uint32_t inv20) { return (e * inv20) >> 20; }

// Product of the R row values modulo 2^64: pairs exactly in 64 bits (|f| < 2^24), then a chain.
template <int R>
__device__ __forceinline__ uint64_t row_product(const int32_t (&f)[R]) {
    uint64_t p = (uint64_t)((int64_t)f[0] * (int64_t)f[1]);
#pragma unroll
    for (int k = 1; k < R / 2; ++k) p *= (uint64_t)((int64_t)f[2 * k] * (int64_t)f[2 * k + 1]);
    return p;
}

template <int R>
__device__ __forceinline__ void add_rows(int32_t (&f)[R], const int32_t *d, bool add) {
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

// This lane's share of V for the leaf of order p (7 <= p <= R) stored row-major at M.
template <int R>
__device__ uint64_t eval_leaf(const uint32_t *M, int p, int lane, int32_t *D, int32_t *base) {
    // delta table D[j][i] = 2 b_ij (Gray column j, padded rows 0) and base_i = 2 b_i,p-1 - R_i
    for (int e = lane; e < (p - 1) * DSTRIDE; e += SW) {
        const int j = e / DSTRIDE, i = e - j * DSTRIDE;
        D[e] = i < p ? 2 * (int32_t)M[i * p + j] : 0;
    }
    if (lane < R) {
        int32_t b = 1;
        if (lane < p) {
            uint32_t rs = 0;
            for (int j = 0; j < p; ++j) rs += M[lane * p + j];
            b = 2 * (int32_t)M[lane * p + p - 1] - (int32_t)rs;
        }
        base[lane] = b;
    }
    wave_sync();
    const int c = p - 7;
    const uint32_t L = 1u << c;
    const uint32_t kfirst = (lane & 1) ? (uint32_t)lane * L + L - 1 : (uint32_t)lane * L;
    const uint32_t s0 = kfirst ^ (kfirst >> 1);
    int32_t f[R];
#pragma unroll
    for (int i = 0; i < R; i += 4) {
        const int4 w = *(const int4 *)(base + i);
        f[i] = w.x;
        f[i + 1] = w.y;
        f[i + 2] = w.z;
        f[i + 3] = w.w;
    }
    for (int j = c; j < p - 1; ++j) {
        const bool in = (s0 >> j) & 1;
        const int32_t *dj = D + j * DSTRIDE;
#pragma unroll
        for (int i = 0; i < R; ++i) f[i] += in ? dj[i] : 0;
    }
    uint64_t acc0 = row_product<R>(f), acc1 = 0;
    for (uint32_t s = 1; s < L; s += 2) {
        add_rows<R>(f, D, ((s >> 1) & 1) == 0);   // odd steps flip Gray column 0
        acc1 += row_product<R>(f);
        if (s + 1 < L) {
            const uint32_t s2 = s + 1;
            const int j = __builtin_ctz(s2);
            add_rows<R>(f, D + j * DSTRIDE, ((s2 >> (j + 1)) & 1) == 0);
            acc0 += row_product<R>(f);
        }
    }
    wave_sync();   // D and base are rewritten by the next leaf
    return (lane & 1) ? acc1 - acc0 : acc0 - acc1;
}

struct SplitCtl {   // word offsets in a control block
    enum { IS_COL, IDX, NP, P0, Q0, CA0, CB0, P1, Q1, CA1, CB1, NEXT };
};

// Child `ch` of the node of order o at M (line and pairs in ctl) written at C (order o - 1).
__device__ void make_child(const uint32_t *M, int o, const uint32_t *ctl, int ch, uint32_t *C, int lane) {
    const uint32_t is_col = uni(ctl[SplitCtl::IS_COL]), line = uni(ctl[SplitCtl::IDX]);
    const uint32_t P = uni(ctl[SplitCtl::P0 + 4 * ch]), Q = uni(ctl[SplitCtl::Q0 + 4 * ch]);
    const uint32_t ca = uni(ctl[SplitCtl::CA0 + 4 * ch]), cb = uni(ctl[SplitCtl::CB0 + 4 * ch]);
    const uint32_t keep = min(P, Q), drop = max(P, Q);
    const uint32_t co = (uint32_t)o - 1, inv = ((1u << 20) + co - 1) / co;
    for (uint32_t e = lane; e < co * co; e += SW) {
        const uint32_t ip = div_small(e, inv), jp = e - ip * co;
        uint32_t v;
        if (!is_col) {   // row `line` deleted, columns P, Q merged at min(P, Q)
            const uint32_t i = ip + (ip >= line), j = jp + (jp >= drop);
            v = j == keep ? ca * M[i * o + Q] + cb * M[i * o + P] : M[i * o + j];
        } else {         // column `line` deleted, rows P, Q merged at min(P, Q)
            const uint32_t i = ip + (ip >= drop), j = jp + (jp >= line);
            v = i == keep ? ca * M[Q * o + j] + cb * M[P * o + j] : M[i * o + j];
        }
        C[e] = v;
    }
    wave_sync();
}

__global__ __launch_bounds__(SW) void hper_split_w64(const JobDesc *__restrict__ jobs,
                                                     const uint32_t *__restrict__ data,
                                                     const uint32_t *__restrict__ queue, uint32_t nqueue,
                                                     int t, int s_leaf, unsigned long long *head,
                                                     JobAcc *__restrict__ accs,
                                                     unsigned long long *__restrict__ stats,
                                                     unsigned long long *__restrict__ cycles) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    const int lane = threadIdx.x;
    uint32_t *slots = lds;
    int32_t *D = (int32_t *)(lds + align4(slot_off(t - 1)));
    int32_t *base = D + SMAX * DSTRIDE;
    uint32_t *ctl_all = (uint32_t *)(base + SMAX);
    auto slot = [&](int o) { return slots + (slot_off(o) - slot_off(SMAX)); };
    uint64_t n_leaves = 0, n_terms = 0, n_splits = 0, n_stops = 0;
    for (;;) {
        const unsigned long long got = atomicAdd(head, lane == 0 ? 1ull : 0ull);
        const uint64_t qi = uni64(got);
        if (qi >= nqueue) break;
        const uint32_t job = uni(queue[qi]);
        const JobDesc jd = jobs[job];
        const int m0 = (int)uni(jd.m);
        const uint32_t *blk = data + (size_t)uni(jd.data_off) * HP_DATA_ALIGN;
        const uint64_t t0 = (uint64_t)clock64();
        // the job as a dense m0 x m0 matrix: Gray columns 0..m0-2, then the fixed column
        uint32_t *R0 = slot(m0);
        for (int e = lane; e < m0 * m0; e += SW) R0[e] = 0;
        wave_sync();
        if (lane < m0 - 1) {
            const uint32_t b = blk[m0 + lane], en = blk[m0 + lane + 1];
            for (uint32_t e = b; e < en; ++e) {
                const uint32_t w = blk[3 * m0 + e];
                R0[(w & 0xffu) * m0 + lane] = w >> 9;
            }
        }
        wave_sync();
        if (lane < m0) {
            int32_t sg = 0;
            for (int g = 0; g < m0 - 1; ++g) sg += (int32_t)R0[lane * m0 + g];
            R0[lane * m0 + m0 - 1] = (uint32_t)((int32_t)blk[lane] + sg);
        }
        wave_sync();
        uint64_t acc = 0;
        int o = m0;
        for (;;) {
            const uint32_t *M = slot(o);
            // Step 1 of H_per: the sparsest line (rows on lanes 0..o-1, columns on 32..32+o-1)
            uint32_t key = 0xffffffffu;
            if (lane < o) {
                uint32_t k = 0;
                for (int j = 0; j < o; ++j) k += M[lane * o + j] != 0;
                key = (k << 6) | (uint32_t)lane;
            } else if (lane >= 32 && lane < 32 + o) {
                uint32_t k = 0;
                for (int i = 0; i < o; ++i) k += M[i * o + (lane - 32)] != 0;
                key = (k << 6) | (uint32_t)lane;
            }
            key = uni(wave_min(key));
            const uint32_t s = key >> 6, is_col = (key >> 5) & 1, line = key & 31;
            bool leaf = false;
            if (s == 0) {
                // dropped: per = 0
            } else if (o <= t || o <= 2 || (int)s >= s_leaf || s > 4) {
                leaf = true;
            } else {
                // the line's nonzeros in increasing index order, pairs, and the bound check
                uint32_t v = 0;
                if (lane < o) v = is_col ? M[lane * o + line] : M[line * o + lane];
                uint64_t nz = __ballot(v != 0);
                const uint64_t all = (1ull << o) - 1;
                const uint32_t zero = (uint32_t)__builtin_ctzll(~nz & all);
                uint32_t pos[4], val[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    pos[k] = zero;
                    val[k] = 0;
                    if ((uint32_t)k < s) {
                        pos[k] = (uint32_t)__builtin_ctzll(nz);
                        nz &= nz - 1;
                        val[k] = uni((uint32_t)__shfl((int)v, (int)pos[k]));
                    }
                }
                const uint32_t np = (s + 1) / 2;
                bool bad = false;
                for (uint32_t ch = 0; ch < np; ++ch) {
                    const uint32_t P = pos[2 * ch], Q = pos[2 * ch + 1];
                    const uint64_t ca = val[2 * ch], cb = val[2 * ch + 1];
                    bool fail = false;
                    if (!is_col) {
                        if (lane < o && (uint32_t)lane != line) {
                            const uint32_t *row = M + lane * o;
                            uint64_t rs = 0;
                            for (int j = 0; j < o; ++j) rs += row[j];
                            const uint64_t mv = ca * row[Q] + cb * row[P];
                            fail = mv >= HP_MAX_ENTRY || rs - row[P] - row[Q] + mv >= HP_MAX_ROWSUM;
                        }
                    } else {
                        uint64_t mv = 0;
                        if (lane < o && (uint32_t)lane != line) {
                            mv = ca * M[Q * o + lane] + cb * M[P * o + lane];
                            fail = mv >= HP_MAX_ENTRY;
                        }
                        const uint64_t merged_sum = wave_sum64(mv);   // every lane takes part
                        fail = fail || merged_sum >= HP_MAX_ROWSUM;
                    }
                    const bool any = __ballot(fail) != 0;
                    bad = bad || any;
                }
                if (bad) {
                    leaf = true;
                    ++n_stops;
                } else {
                    uint32_t *ctl = ctl_all + o * CTL;
                    if (lane == 0) {
                        ctl[SplitCtl::IS_COL] = is_col;
                        ctl[SplitCtl::IDX] = line;
                        ctl[SplitCtl::NP] = np;
                        ctl[SplitCtl::P0] = pos[0];
                        ctl[SplitCtl::Q0] = pos[1];
                        ctl[SplitCtl::CA0] = val[0];
                        ctl[SplitCtl::CB0] = val[1];
                        ctl[SplitCtl::P1] = pos[2];
                        ctl[SplitCtl::Q1] = pos[3];
                        ctl[SplitCtl::CA1] = val[2];
                        ctl[SplitCtl::CB1] = val[3];
                        ctl[SplitCtl::NEXT] = 0;
                    }
                    wave_sync();
                    make_child(M, o, ctl, 0, slot(o - 1), lane);
                    ++n_splits;
                    --o;
                    continue;
                }
            }
            if (leaf) {
                uint64_t v;
                if (o <= 12) v = eval_leaf<12>(M, o, lane, D, base);
                else if (o <= 16) v = eval_leaf<16>(M, o, lane, D, base);
                else v = eval_leaf<20>(M, o, lane, D, base);
                const int sh = m0 - o;
                v <<= sh;
                acc += (sh & 1) ? (uint64_t)0 - v : v;
                ++n_leaves;
                n_terms += 1ull << (o - 1);
            }
            // back up to the nearest node on the path with a child left
            int up = o + 1;
            for (; up <= m0; ++up) {
                uint32_t *ctl = ctl_all + up * CTL;
                const uint32_t nx = uni(ctl[SplitCtl::NEXT]) + 1;
                if (nx < uni(ctl[SplitCtl::NP])) {
                    if (lane == 0) ctl[SplitCtl::NEXT] = nx;
                    wave_sync();
                    make_child(slot(up), up, ctl, (int)nx, slot(up - 1), lane);
                    break;
                }
            }
            if (up > m0) break;
            o = up - 1;
        }
        const uint64_t total = wave_sum64(acc);
        if (lane == 0) {
            accs[job].l[0] = total;
            if (cycles) cycles[job] = (unsigned long long)((uint64_t)clock64() - t0);
        }
    }
    if (lane == 0) {
        atomicAdd(stats + 0, (unsigned long long)n_leaves);
        atomicAdd(stats + 1, (unsigned long long)n_terms);
        atomicAdd(stats + 2, (unsigned long long)n_splits);
        atomicAdd(stats + 3, (unsigned long long)n_stops);
    }
}

}  // namespace

size_t split_lds_bytes(int t) { return (size_t)region_words(t) * sizeof(uint32_t); }

hipError_t launch_split_w64(const JobDesc *jobs, const uint32_t *data, const uint32_t *queue, uint32_t n,
                            int t, int s_leaf, unsigned long long *head, JobAcc *accs,
                            unsigned long long *stats, unsigned long long *cycles, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (t < HP_SPLIT_MIN_T || t >= HP_SPLIT_MAX_M) return hipErrorInvalidValue;
    const size_t lds = split_lds_bytes(t);
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, hper_split_w64, SW, lds);
    if (e != hipSuccess) return e;
    uint64_t grid = (uint64_t)cus * (uint64_t)(per_cu > 0 ? per_cu : 1);
    if (grid > n) grid = n;
    hipLaunchKernelGGL(hper_split_w64, dim3((uint32_t)grid), dim3(SW), lds, s, jobs, data, queue, n, t, s_leaf,
                       head, accs, stats, cycles);
    return hipGetLastError();
}

}  // namespace hp
