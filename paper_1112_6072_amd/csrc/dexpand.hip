// Device expansion: Algorithm H_per's splitting (Section 2.1) and the pre-expansion of
// Algorithm PH (Step 2, Section 2.2) run on the GPU, one tree level at a time, from the input
// matrix down to sub-matrix jobs of a target order, which the device continuation of H_per then
// finishes. Every split lowers the order by one, so a level holds nodes of one order.
//
// A level is expanded chunk by chunk in three steps:
//   1. plan: one wave per node finds its sparsest line (Step 1 of H_per: the fewest nonzeros
//      s over rows and columns; ties: rows first, then the lowest index) and its child count
//      ceil(s/2) (0 drops the node: per = 0); every child needs at most the parent's words;
//   2. an exclusive scan of (children, words) gives each node's output place;
//   3. write: one wave per node writes its children by expansion (2) along that line:
//      consecutive nonzeros of the line are paired and each pair's two columns (rows, for a
//      column line) merged with crossed weights, the line deleted; an odd last nonzero is
//      paired at weight 0 with the lowest zero of the line. Lanes own rows. A child entry
//      >= 2^22 or row sum >= 2^24 is reported (the limits every job keeps).
// Nodes whose sparsest line has five or more nonzeros are split the same way (ceil(s/2)
// children): above the job order R-NW cannot take them, and the expansion is an identity.
// Modular mode (a prime p < 2^18 per problem, with n (p - 1) < 2^24): every merged entry is
// reduced modulo its problem's p, so entries stay below p and row sums below 2^24; the tree
// then computes per(A) mod p (the permanental polynomial's evaluations, and per(A) past the
// exact rings, by residues).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hperm_internal.h"
#include "kernels.h"

namespace hp {
namespace {

constexpr int WV = 64;
constexpr int BLK = 256;                 // 4 waves, one node each
constexpr int MAXO = HP_MAX_N;           // largest node order (two rows per lane)

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    return (uint64_t)uni((uint32_t)x) | ((uint64_t)uni((uint32_t)(x >> 32)) << 32);
}
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    for (int o = 32; o; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}
__device__ __forceinline__ float wave_sumf(float v) {
    for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
// Exclusive prefix sum over the lanes; *total receives the sum.
__device__ __forceinline__ uint32_t wave_excl(uint32_t v, int lane, uint32_t *total) {
    uint32_t x = v;
    for (int o = 1; o < WV; o <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)x, o);
        if (lane >= o) x += u;
    }
    *total = (uint32_t)__shfl((int)x, WV - 1);
    return x - v;
}

// The modulus of modular mode (p = 0: exact arithmetic), with its FP64 reciprocal.
struct Modulus {
    uint32_t p;
    double pd, pinv;
};
__device__ __forceinline__ Modulus modulus(uint32_t p) { return Modulus{p, (double)p, p ? 1.0 / (double)p : 0.0}; }

// A merged entry in the expansion's arithmetic: exact, or reduced modulo p in modular mode
// (p > 0: per(A) modulo p, every entry kept below p). There v = ca q + cb p < 2^37, exact in
// FP64: v - floor(v / p) p with the quotient off by at most one, corrected.
__device__ __forceinline__ uint64_t merged(uint64_t v, const Modulus &m) {
    if (!m.p) return v;
    const double x = (double)v;
    double r = __builtin_fma(-floor(x * m.pinv), m.pd, x);
    r = r < 0.0 ? r + m.pd : r;
    r = r >= m.pd ? r - m.pd : r;
    return (uint64_t)r;
}

// A node's rows: lane holds rows lane and lane + 64 (length, first entry index).
struct Rows {
    uint32_t len[2], start[2];
};

__device__ __forceinline__ Rows node_rows(const uint32_t *node, int o, int lane) {
    Rows r;
    uint32_t tot0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        r.len[h] = i < o ? (node[4 + i / 4] >> (8 * (i & 3))) & 0xffu : 0u;
    }
    r.start[0] = wave_excl(r.len[0], lane, &tot0);
    uint32_t tot1;
    r.start[1] = tot0 + wave_excl(r.len[1], lane, &tot1);
    return r;
}

// Value of line i (two per lane: lanes hold lines lane and lane + 64) from the lane holding it.
__device__ __forceinline__ uint32_t pick(const uint32_t (&v)[2], uint32_t i) {
    const uint32_t a = (uint32_t)__shfl((int)v[0], (int)(i & 63)), b = (uint32_t)__shfl((int)v[1], (int)(i & 63));
    return i >= 64 ? b : a;
}

__device__ __forceinline__ const uint32_t *node_entries(const uint32_t *node, int o) { return node + 4 + (o + 3) / 4; }

// Step 1 of H_per: the key (s << 9) | (is_col << 8) | index of the sparsest line. hist is the
// wave's LDS column-count array (MAXO words).
__device__ __forceinline__ uint32_t line_key(const uint32_t *node, int o, const Rows &r, uint32_t *hist, int lane) {
    const uint32_t *ent = node_entries(node, o);
    for (int j = lane; j < MAXO; j += WV) hist[j] = 0;
    wave_sync();
#pragma unroll
    for (int h = 0; h < 2; ++h)
        for (uint32_t e = 0; e < r.len[h]; ++e) atomicAdd(hist + (ent[r.start[h] + e] & 0xffu), 1u);
    wave_sync();
    uint32_t best = 0xffffffffu;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        if (i < o) {
            best = min(best, (r.len[h] << 9) | (uint32_t)i);
            best = min(best, (hist[i] << 9) | 256u | (uint32_t)i);
        }
    }
    return uni(wave_min(best));
}

__device__ __forceinline__ uint32_t node_words_of(const uint32_t *node) {
    const uint32_t h0 = node[0];
    return hp_node_words((int)(h0 & 0xffu), (int)(h0 >> 8));
}

__global__ __launch_bounds__(BLK) void dexp_plan(const uint32_t *__restrict__ lvl, const uint64_t *__restrict__ off,
                                                 uint64_t first, uint32_t n, uint32_t *__restrict__ key_out,
                                                 uint64_t *__restrict__ packed) {
    __shared__ uint32_t hist_all[BLK / WV][MAXO];
    const int lane = threadIdx.x & (WV - 1), wv = threadIdx.x / WV;
    const uint32_t k = blockIdx.x * (BLK / WV) + wv;
    if (k >= n) return;
    const uint32_t *node = lvl + uni64(off[first + k]);
    const int o = (int)(uni(node[0]) & 0xffu);
    const Rows r = node_rows(node, o, lane);
    const uint32_t key = line_key(node, o, r, hist_all[wv], lane);
    if (lane == 0) {
        const uint32_t s = key >> 9;
        const uint64_t np = (s + 1) / 2;
        key_out[k] = key;
        packed[k] = (np << 36) | (np * node_words_of(node));
    }
}

// ------------------------------------------------------------------ exclusive scan (u64)
constexpr int SCAN_PER = 4;                      // elements per thread
constexpr int SCAN_TILE = BLK * SCAN_PER;

__device__ __forceinline__ uint64_t block_excl(uint64_t v, uint64_t *sh, uint64_t *total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < BLK; o <<= 1) {
        const uint64_t u = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += u;
        __syncthreads();
    }
    *total = sh[BLK - 1];
    const uint64_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(BLK) void scan_tiles(const uint64_t *__restrict__ in, uint32_t n, uint64_t *__restrict__ sums) {
    __shared__ uint64_t sh[BLK];
    uint64_t v = 0;
    for (int q = 0; q < SCAN_PER; ++q) {
        const uint64_t i = (uint64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER + q;
        if (i < n) v += in[i];
    }
    uint64_t tot;
    block_excl(v, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One block: exclusive scan of the tile sums in place; *grand receives their total.
__global__ __launch_bounds__(BLK) void scan_sums(uint64_t *__restrict__ sums, uint32_t ntiles, uint64_t *__restrict__ grand) {
    __shared__ uint64_t sh[BLK];
    uint64_t carry = 0;
    for (uint32_t b = 0; b < ntiles; b += BLK) {
        const uint32_t i = b + threadIdx.x;
        const uint64_t v = i < ntiles ? sums[i] : 0;
        uint64_t tot;
        const uint64_t ex = block_excl(v, sh, &tot);
        if (i < ntiles) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *grand = carry;
}

__global__ __launch_bounds__(BLK) void scan_apply(const uint64_t *__restrict__ in, uint32_t n,
                                                  const uint64_t *__restrict__ sums, uint64_t *__restrict__ out) {
    __shared__ uint64_t sh[BLK];
    uint64_t v[SCAN_PER], s = 0;
    for (int q = 0; q < SCAN_PER; ++q) {
        const uint64_t i = (uint64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER + q;
        v[q] = i < n ? in[i] : 0;
        s += v[q];
    }
    uint64_t tot;
    uint64_t ex = block_excl(s, sh, &tot) + sums[blockIdx.x];
    for (int q = 0; q < SCAN_PER; ++q) {
        const uint64_t i = (uint64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER + q;
        if (i < n) out[i] = ex;
        ex += v[q];
    }
}

// ------------------------------------------------------------------ children
// The c-th pair of the line: positions P (coefficient of the merge: cb) and Q (coefficient ca),
// the merge being ca * y_Q + cb * y_P as in expansion (2) (y_P the line through the first
// nonzero of the pair).
struct Pair {
    uint32_t P, Q, ca, cb;
};

// Row line r: its entries are the pairs' positions in column order.
__device__ __forceinline__ Pair row_pair(const uint32_t *ent, uint32_t rstart, uint32_t rlen, int o, uint32_t c) {
    Pair pr;
    const uint32_t w0 = uni(ent[rstart + 2 * c]);
    pr.P = w0 & 0xffu;
    pr.ca = w0 >> 8;
    if (2 * c + 1 < rlen) {
        const uint32_t w1 = uni(ent[rstart + 2 * c + 1]);
        pr.Q = w1 & 0xffu;
        pr.cb = w1 >> 8;
    } else {   // the lowest column that is zero in the row (or the lowest other column)
        uint32_t z = 0xffffffffu;
        for (uint32_t e = 0; e < rlen && z == 0xffffffffu; ++e)
            if ((uni(ent[rstart + e]) & 0xffu) != e) z = e;
        if (z == 0xffffffffu) z = rlen < (uint32_t)o ? rlen : (pr.P == 0 ? 1u : 0u);
        pr.Q = z;
        pr.cb = 0;
    }
    return pr;
}

// The k-th set bit (k >= 0) of the 128-bit mask (lo, hi).
__device__ __forceinline__ uint32_t nth_bit(uint64_t lo, uint64_t hi, uint32_t k) {
    const uint32_t nlo = (uint32_t)__popcll(lo);
    uint64_t m = k < nlo ? lo : hi;
    uint32_t kk = k < nlo ? k : k - nlo;
    for (uint32_t q = 0; q < kk; ++q) m &= m - 1;
    return (uint32_t)__builtin_ctzll(m) + (k < nlo ? 0u : 64u);
}

// The children of one node (its words at `node`, read from LDS when staged) by expansion (2)
// along the line of `key`. With a staging buffer `cst`, each child is built there and copied
// to its place in `out` with coalesced stores; else it is written to `out` directly.
__device__ __forceinline__ void write_children(const uint32_t *node, uint32_t key, uint64_t child_idx, uint64_t wbase,
                                               uint32_t *lenb, uint32_t *cst, uint32_t *__restrict__ out,
                                               uint64_t *__restrict__ out_off, unsigned long long *__restrict__ flags,
                                               const Modulus &modp, int lane) {
    const uint32_t h0 = uni(node[0]);
    const int o = (int)(h0 & 0xffu);
    const float pbound = __uint_as_float(uni(node[1]));
    const uint32_t problem = uni(node[2]);
    const uint32_t s = key >> 9, is_col = (key >> 8) & 1u, line = key & 0xffu;
    const uint32_t np = (s + 1) / 2;
    const uint32_t pw = hp_node_words(o, (int)(h0 >> 8));
    const uint32_t *ent = node_entries(node, o);
    const Rows r = node_rows(node, o, lane);
    // the line's nonzeros: a row line reads its entries; a column line finds its rows
    uint32_t rstart = 0, rlen = 0;
    uint64_t cl_lo = 0, cl_hi = 0;   // rows holding the column line
    uint32_t cval[2] = {0, 0};       // this lane's rows' entries in the column line
    if (!is_col) {
        rstart = uni((uint32_t)pick(r.start, line));
        rlen = uni((uint32_t)pick(r.len, line));
    } else {
#pragma unroll
        for (int h = 0; h < 2; ++h)
            for (uint32_t e = 0; e < r.len[h]; ++e) {
                const uint32_t w = ent[r.start[h] + e];
                if ((w & 0xffu) == line) cval[h] = w >> 8;
            }
        cl_lo = __ballot(cval[0] != 0);
        cl_hi = __ballot(cval[1] != 0);
    }
    const uint32_t co = (uint32_t)o - 1;
    bool bad = false;
    for (uint32_t c = 0; c < np; ++c) {
        Pair pr;
        if (!is_col) {
            pr = row_pair(ent, rstart, rlen, o, c);
        } else {
            pr.P = nth_bit(cl_lo, cl_hi, 2 * c);
            pr.ca = uni((uint32_t)pick(cval, pr.P));
            if (2 * c + 1 < s) {
                pr.Q = nth_bit(cl_lo, cl_hi, 2 * c + 1);
                pr.cb = uni((uint32_t)pick(cval, pr.Q));
            } else {   // the lowest row that is zero in the column (or the lowest other row)
                const uint64_t vlo = o >= 64 ? ~0ull : ((1ull << o) - 1);
                const uint64_t vhi = o > 64 ? (o >= 128 ? ~0ull : ((1ull << (o - 64)) - 1)) : 0ull;
                const uint64_t zl = ~cl_lo & vlo, zh = ~cl_hi & vhi;
                pr.Q = zl ? (uint32_t)__builtin_ctzll(zl) : zh ? 64u + (uint32_t)__builtin_ctzll(zh) : (pr.P == 0 ? 1u : 0u);
                pr.cb = 0;
            }
        }
        const uint32_t keep = min(pr.P, pr.Q), drop = max(pr.P, pr.Q);
        uint32_t *const Cg = out + wbase + (uint64_t)c * pw;
        uint32_t *C = cst ? cst : Cg;
        // pass 1: each lane's output rows, their lengths and sums
        uint32_t olen[2] = {0, 0}, orow[2] = {0xffffffffu, 0xffffffffu};
        uint64_t osum[2] = {0, 0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t i = (uint32_t)lane + 64u * h;
            if (i >= (uint32_t)o) continue;
            if (!is_col) {
                if (i == line) continue;
                orow[h] = i - (i > line);
                uint64_t ap = 0, aq = 0, rest = 0;
                uint32_t cnt = 0;
                for (uint32_t e = 0; e < r.len[h]; ++e) {
                    const uint32_t w = ent[r.start[h] + e], j = w & 0xffu, v = w >> 8;
                    if (j == pr.P) ap = v;
                    else if (j == pr.Q) aq = v;
                    else {
                        ++cnt;
                        rest += v;
                    }
                }
                const uint64_t mv = merged((uint64_t)pr.ca * aq + (uint64_t)pr.cb * ap, modp);
                bad = bad || mv >= HP_MAX_ENTRY;
                olen[h] = cnt + (mv != 0);
                osum[h] = rest + mv;
            } else {
                if (i == drop) continue;
                orow[h] = i - (i > drop);
                if (i != keep) {
                    uint64_t rest = 0;
                    uint32_t cnt = 0;
                    for (uint32_t e = 0; e < r.len[h]; ++e) {
                        const uint32_t w = ent[r.start[h] + e];
                        if ((w & 0xffu) != line) {
                            ++cnt;
                            rest += w >> 8;
                        }
                    }
                    olen[h] = cnt;
                    osum[h] = rest;
                }   // row keep (ca * row Q + cb * row P, without the column line): below
            }
            bad = bad || osum[h] >= HP_MAX_ROWSUM;
        }
        // the merged row of a column split: read by the lane owning row keep; the starts and
        // lengths of rows P and Q come from their owners
        uint32_t qs = 0, ql = 0, ps = 0, plen = 0;
        if (is_col) {
            qs = uni((uint32_t)pick(r.start, pr.Q));
            ql = uni((uint32_t)pick(r.len, pr.Q));
            ps = uni((uint32_t)pick(r.start, pr.P));
            plen = uni((uint32_t)pick(r.len, pr.P));
            if ((uint32_t)lane == (keep & 63)) {
                const int h = keep >> 6;
                uint32_t a = 0, b = 0, cnt = 0;
                uint64_t sum = 0;
                while (a < ql || b < plen) {
                    const uint32_t wq = a < ql ? ent[qs + a] : 0xffffffffu, wp = b < plen ? ent[ps + b] : 0xffffffffu;
                    const uint32_t jq = a < ql ? (wq & 0xffu) : 0x1ffu, jp = b < plen ? (wp & 0xffu) : 0x1ffu;
                    const uint32_t j = min(jq, jp);
                    uint64_t mv = 0;
                    if (jq == j) {
                        mv += (uint64_t)pr.ca * (wq >> 8);
                        ++a;
                    }
                    if (jp == j) {
                        mv += (uint64_t)pr.cb * (wp >> 8);
                        ++b;
                    }
                    mv = merged(mv, modp);
                    if (j == line || mv == 0) continue;
                    bad = bad || mv >= HP_MAX_ENTRY;
                    ++cnt;
                    sum += mv;
                }
                if (h) {
                    olen[1] = cnt;
                    osum[1] = sum;
                } else {
                    olen[0] = cnt;
                    osum[0] = sum;
                }
                bad = bad || sum >= HP_MAX_ROWSUM;
            }
        }
        // output row order = input row order without the deleted row
        uint32_t tot0, tot1;
        const uint32_t ostart0 = wave_excl(olen[0], lane, &tot0);
        const uint32_t ostart1 = tot0 + wave_excl(olen[1], lane, &tot1);
        const uint32_t onnz = tot0 + tot1;
        const uint32_t ostart[2] = {ostart0, ostart1};
        // the child's bound: the parent's, or its own product of row sums
        float lb = 0.0f;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (orow[h] != 0xffffffffu) lb += osum[h] ? __log2f((float)osum[h]) : -1e30f;
        lb = wave_sumf(lb) + 1e-3f;
        const float cbound = fminf(pbound, lb);
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (orow[h] != 0xffffffffu) lenb[orow[h]] = olen[h];
        wave_sync();
        uint32_t *cent = C + 4 + (co + 3) / 4;
        for (uint32_t q = (uint32_t)lane; q < (co + 3) / 4; q += WV) {
            uint32_t wd = 0;
            for (uint32_t b = 0; b < 4; ++b)
                if (4 * q + b < co) wd |= (lenb[4 * q + b] & 0xffu) << (8 * b);
            C[4 + q] = wd;
        }
        const uint32_t cwords = hp_node_words((int)co, (int)onnz);
        if (lane == 0) {
            C[0] = co | (onnz << 8);
            C[1] = __float_as_uint(cbound < -1e29f ? -INFINITY : cbound);
            C[2] = problem;
            C[3] = 0;
            out_off[child_idx + c] = wbase + (uint64_t)c * pw;
        }
        // pass 2: the entries
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t i = (uint32_t)lane + 64u * h;
            if (orow[h] == 0xffffffffu) continue;
            uint32_t *dst = cent + ostart[h];
            if (!is_col) {
                uint64_t ap = 0, aq = 0;
                for (uint32_t e = 0; e < r.len[h]; ++e) {
                    const uint32_t w = ent[r.start[h] + e], j = w & 0xffu;
                    if (j == pr.P) ap = w >> 8;
                    if (j == pr.Q) aq = w >> 8;
                }
                // presence from the full 64-bit value, as in the row lengths of the plan above:
                // an out-of-range value (flagged) is stored truncated but never changes the
                // node's shape
                const uint64_t mv64 = merged((uint64_t)pr.ca * aq + (uint64_t)pr.cb * ap, modp);
                const uint32_t mv = (uint32_t)mv64;
                bool merged = false;
                uint32_t q = 0;
                for (uint32_t e = 0; e < r.len[h]; ++e) {
                    const uint32_t w = ent[r.start[h] + e], j = w & 0xffu;
                    if (j == pr.P || j == pr.Q) continue;
                    if (!merged && j > keep) {
                        if (mv64) dst[q++] = (mv << 8) | keep;
                        merged = true;
                    }
                    dst[q++] = (w & ~0xffu) | (j - (j > drop));
                }
                if (!merged && mv64) dst[q++] = (mv << 8) | keep;
            } else if (i != keep) {
                uint32_t q = 0;
                for (uint32_t e = 0; e < r.len[h]; ++e) {
                    const uint32_t w = ent[r.start[h] + e], j = w & 0xffu;
                    if (j == line) continue;
                    dst[q++] = (w & ~0xffu) | (j - (j > line));
                }
            } else {
                uint32_t a = 0, b = 0, q = 0;
                while (a < ql || b < plen) {
                    const uint32_t wq = a < ql ? ent[qs + a] : 0xffffffffu, wp = b < plen ? ent[ps + b] : 0xffffffffu;
                    const uint32_t jq = a < ql ? (wq & 0xffu) : 0x1ffu, jp = b < plen ? (wp & 0xffu) : 0x1ffu;
                    const uint32_t j = min(jq, jp);
                    uint64_t mv = 0;
                    if (jq == j) {
                        mv += (uint64_t)pr.ca * (wq >> 8);
                        ++a;
                    }
                    if (jp == j) {
                        mv += (uint64_t)pr.cb * (wp >> 8);
                        ++b;
                    }
                    mv = merged(mv, modp);
                    if (j == line || mv == 0) continue;
                    dst[q++] = ((uint32_t)mv << 8) | (j - (j > line));
                }
            }
        }
        wave_sync();   // lenb (and the staging buffer) are rewritten by the next child
        if (cst) {
            for (uint32_t q = (uint32_t)lane; q < cwords; q += WV) Cg[q] = cst[q];
            wave_sync();
        }
    }
    if (__ballot(bad) != 0 && lane == 0) atomicOr(flags, 1ull);
}

// Nodes up to this many words are staged in LDS (a cubic graph on 128 vertices takes about 420).
constexpr int NODE_LDS = 512;

__global__ __launch_bounds__(BLK) void dexp_write(const uint32_t *__restrict__ lvl, const uint64_t *__restrict__ off,
                                                  uint64_t first, uint32_t n, const uint32_t *__restrict__ keys,
                                                  const uint64_t *__restrict__ place,
                                                  uint32_t *__restrict__ out, uint64_t *__restrict__ out_off,
                                                  unsigned long long *__restrict__ flags,
                                                  const uint32_t *__restrict__ primes) {
    __shared__ uint32_t len_all[BLK / WV][MAXO];
    __shared__ __attribute__((aligned(16))) uint32_t node_all[BLK / WV][NODE_LDS];
    __shared__ __attribute__((aligned(16))) uint32_t child_all[BLK / WV][NODE_LDS];
    const int lane = threadIdx.x & (WV - 1), wv = threadIdx.x / WV;
    const uint32_t k = blockIdx.x * (BLK / WV) + wv;
    if (k >= n) return;
    const uint32_t key = uni(keys[k]);
    if ((key >> 9) == 0) return;   // a line without nonzeros: no children (per = 0)
    const uint32_t *node = lvl + uni64(off[first + k]);
    const uint32_t h0 = uni(node[0]);
    const uint32_t pw = hp_node_words((int)(h0 & 0xffu), (int)(h0 >> 8));
    const Modulus modp = modulus(primes ? uni(primes[uni(node[2])]) : 0u);   // the node's problem's prime
    const uint64_t pl = uni64(place[k]);
    const uint64_t child_idx = pl >> 36, wbase = pl & ((1ull << 36) - 1);
    if (pw <= (uint32_t)NODE_LDS) {   // coalesced copy in, children built in LDS, copied out
        uint32_t *nb = node_all[wv];
        for (uint32_t q = (uint32_t)lane; q < pw; q += WV) nb[q] = node[q];
        wave_sync();
        write_children(nb, key, child_idx, wbase, len_all[wv], child_all[wv], out, out_off, flags, modp, lane);
    } else {
        write_children(node, key, child_idx, wbase, len_all[wv], nullptr, out, out_off, flags, modp, lane);
    }
}

}  // namespace

hipError_t launch_dexp_plan(const uint32_t *lvl, const uint64_t *off, uint64_t first, uint32_t n, uint32_t *keys,
                            uint64_t *packed, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = (n + BLK / WV - 1) / (BLK / WV);
    hipLaunchKernelGGL(dexp_plan, dim3(blocks), dim3(BLK), 0, s, lvl, off, first, n, keys, packed);
    return hipGetLastError();
}

size_t dexp_scan_tiles(uint32_t n) { return ((size_t)n + SCAN_TILE - 1) / SCAN_TILE; }

hipError_t launch_dexp_scan(const uint64_t *in, uint32_t n, uint64_t *tile_sums, uint64_t *out, uint64_t *grand,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t tiles = (uint32_t)dexp_scan_tiles(n);
    hipLaunchKernelGGL(scan_tiles, dim3(tiles), dim3(BLK), 0, s, in, n, tile_sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(BLK), 0, s, tile_sums, tiles, grand);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_apply, dim3(tiles), dim3(BLK), 0, s, in, n, (const uint64_t *)tile_sums, out);
    return hipGetLastError();
}

hipError_t launch_dexp_write(const uint32_t *lvl, const uint64_t *off, uint64_t first, uint32_t n, const uint32_t *keys,
                             const uint64_t *place, uint32_t *out, uint64_t *out_off, unsigned long long *flags,
                             const uint32_t *primes, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = (n + BLK / WV - 1) / (BLK / WV);
    hipLaunchKernelGGL(dexp_write, dim3(blocks), dim3(BLK), 0, s, lvl, off, first, n, keys, place, out, out_off, flags,
                       primes);
    return hipGetLastError();
}

}  // namespace hp
