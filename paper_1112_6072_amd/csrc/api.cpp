// C ABI of libhperm and the host side of the GPU pipeline: device buffers, job upload,
// KKLLL keys, the job order of the device queue (Step 3 of Algorithm PH, improved form of
// Section 3.3), R-NW launches and the exact recombination of job values into per(A)
// (Step 4 of Algorithm PH).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "ctx.h"
#include "expand.h"
#include "kernels.h"

using namespace hp;

namespace hp {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

uint64_t next_jobs_id() {
    static std::atomic<uint64_t> ctr{1};
    return ctr.fetch_add(1);
}

hperm_status set_error(Dev *c, hperm_status s, const std::string &msg) {
    if (c) c->last_error = msg;
    return s;
}

hperm_status set_error(hperm_ctx *c, hperm_status s, const std::string &msg) {
    if (c) c->dev.last_error = msg;
    return s;
}

hperm_status hip_check(Dev *c, hipError_t e, const char *what) {
    if (e == hipSuccess) return HPERM_OK;
    if (e == hipErrorOutOfMemory)
        return set_error(c, HPERM_E_NOMEM, std::string(what) + ": " + hipGetErrorString(e));
    return set_error(c, HPERM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

ExpandParams expand_params(const hperm_opts &o) {
    ExpandParams p;
    p.m_cut = o.m_cut;
    p.m_cap = o.m_cap;
    p.s_leaf = o.s_leaf;
    p.arith = o.arith;
    p.chunk_log2 = o.chunk_log2;
    p.threads = o.host_threads;
    p.max_bytes = (size_t)(o.max_table_mib > 0 ? o.max_table_mib : 4096) << 20;
    return p;
}

static const size_t kAlign = 256;
static size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Make buffer id hold at least `bytes`. With an arena, every buffer is a slice of it and a
// growing buffer re-lays out all slices (their contents are transient per call).
hperm_status ensure_buf(Dev *c, BufId id, size_t bytes) {
    bytes = align_up(std::max<size_t>(bytes, kAlign));
    DevBuf &b = c->buf[id];
    if (b.ptr && b.cap >= bytes) return HPERM_OK;
    if (c->arena) {
        size_t total = 0;
        for (int k = 0; k < B_COUNT; ++k) total += (k == id) ? bytes : c->buf[k].cap;
        if (total > c->arena_bytes) {
            c->arena_required = total;
            return set_error(c, HPERM_E_NOMEM, "the caller's arena is too small");
        }
        size_t off = 0;
        bool moved = false;
        for (int k = 0; k < B_COUNT; ++k) {
            const size_t cap = (k == id) ? bytes : c->buf[k].cap;
            void *p = cap ? (char *)c->arena + off : nullptr;
            if ((k == B_DESC || k == B_DATA) && p != c->buf[k].ptr) moved = true;
            c->buf[k].ptr = p;
            c->buf[k].cap = cap;
            c->buf[k].owned = false;
            off += cap;
        }
        if (moved) c->resident_jobs = 0;
        c->resident_list = 0;
        return HPERM_OK;
    }
    if (b.ptr && b.owned) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_check(c, e, "hipStreamSynchronize");
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.cap = 0;
    }
    if (id == B_DESC || id == B_DATA) c->resident_jobs = 0;
    if (id == B_LIST) c->resident_list = 0;
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        c->arena_required = bytes;
        return hip_check(c, e, "hipMalloc");
    }
    b.cap = bytes;
    b.owned = true;
    return HPERM_OK;
}

hperm_status upload_jobs(Dev *c, hperm_jobs *j) {
    if (c->resident_jobs == j->id && j->id != 0) return HPERM_OK;
    const size_t nd = j->tab.desc.size();
    const size_t nw = j->tab.data.size() + 64;   // padding: lanes may read a few words past a block
    hperm_status s = ensure_buf(c, B_DESC, nd * sizeof(JobDesc));
    if (s) return s;
    s = ensure_buf(c, B_DATA, nw * sizeof(uint32_t));
    if (s) return s;
    s = ensure_buf(c, B_BOUND, nd * sizeof(float));
    if (s) return s;
    if (nd) {
        s = hip_check(c, hipMemcpyAsync(c->buf[B_DESC].ptr, j->tab.desc.data(), nd * sizeof(JobDesc),
                                        hipMemcpyHostToDevice, c->stream), "upload jobs");
        if (s) return s;
        s = hip_check(c, hipMemcpyAsync(c->buf[B_DATA].ptr, j->tab.data.data(),
                                        j->tab.data.size() * sizeof(uint32_t),
                                        hipMemcpyHostToDevice, c->stream), "upload job data");
        if (s) return s;
        static const uint32_t zeros[64] = {0};
        s = hip_check(c, hipMemcpyAsync((char *)c->buf[B_DATA].ptr + j->tab.data.size() * 4, zeros,
                                        sizeof(zeros), hipMemcpyHostToDevice, c->stream),
                      "pad job data");
        if (s) return s;
        // the proven bounds as floats rounded up (the device continuation of H_per admits a
        // leaf to its 64-bit walk by them); kept with the table until it is uploaded again
        if (j->fbound.size() != nd) {
            j->fbound.resize(nd);
            for (size_t k = 0; k < nd; ++k) {
                float f = (float)j->tab.log2_bound[k];
                if ((double)f < j->tab.log2_bound[k]) f = std::nextafter(f, INFINITY);
                j->fbound[k] = f;
            }
        }
        s = hip_check(c, hipMemcpyAsync(c->buf[B_BOUND].ptr, j->fbound.data(), nd * sizeof(float),
                                        hipMemcpyHostToDevice, c->stream), "upload job bounds");
        if (s) return s;
    }
    c->resident_jobs = j->id;
    return HPERM_OK;
}

hperm_status estimate_jobs(Dev *c, hperm_jobs *j, int trials, uint64_t seed) {
    if (trials < 1 || trials > 4096) return set_error(c, HPERM_E_INVALID, "trials must be in [1, 4096]");
    const size_t nd = j->tab.desc.size();
    j->keys.assign(nd, -INFINITY);
    if (nd == 0) {
        j->has_keys = true;
        return HPERM_OK;
    }
    if (nd >= (1u << 28)) return set_error(c, HPERM_E_INVALID, "too many jobs for the estimator");
    hperm_status s = upload_jobs(c, j);
    if (s) return s;
    s = ensure_buf(c, B_KEYS, nd * sizeof(float));
    if (s) return s;
    s = ensure_buf(c, B_LIST, nd * sizeof(uint32_t));
    if (s) return s;
    if (c->resident_jobs != j->id) {   // the arena was re-laid out: upload again
        s = upload_jobs(c, j);
        if (s) return s;
    }
    // jobs grouped by order bucket (one counting pass, once per job table), natural order
    // inside a bucket; uploaded when not already in place
    if (j->elist.size() != nd) {
        std::vector<size_t> &off = j->eoff;
        off.assign(HP_EST_BUCKETS + 1, 0);
        for (size_t k = 0; k < nd; ++k) off[est_bucket_of(j->tab.desc[k].m) + 1]++;
        for (int b = 0; b < HP_EST_BUCKETS; ++b) off[b + 1] += off[b];
        std::vector<size_t> pos(off.begin(), off.end() - 1);
        j->elist.resize(nd);
        for (size_t k = 0; k < nd; ++k) j->elist[pos[est_bucket_of(j->tab.desc[k].m)]++] = (uint32_t)k;
    }
    const std::vector<size_t> &off = j->eoff;
    if (c->resident_list != j->id || c->resident_list_ptr != c->buf[B_LIST].ptr || j->id == 0) {
        s = hip_check(c, hipMemcpyAsync(c->buf[B_LIST].ptr, j->elist.data(), nd * 4, hipMemcpyHostToDevice,
                                        c->stream), "upload estimate list");
        if (s) return s;
        c->resident_list = j->id;
        c->resident_list_ptr = c->buf[B_LIST].ptr;
    }
    for (int b = 0; b < HP_EST_BUCKETS; ++b) {
        const uint32_t n = (uint32_t)(off[b + 1] - off[b]);
        if (!n) continue;
        s = hip_check(c, launch_estimate(b, (const JobDesc *)c->buf[B_DESC].ptr,
                                         (const uint32_t *)c->buf[B_DATA].ptr,
                                         (const uint32_t *)c->buf[B_LIST].ptr + off[b], n, trials, seed,
                                         (float *)c->buf[B_KEYS].ptr, c->stream),
                      "kkl_estimate launch");
        if (s) return s;
    }
    s = hip_check(c, hipMemcpyAsync(j->keys.data(), c->buf[B_KEYS].ptr, nd * sizeof(float),
                                    hipMemcpyDeviceToHost, c->stream), "download keys");
    if (s) return s;
    s = hip_check(c, hipStreamSynchronize(c->stream), "estimate");
    if (s) return s;
    j->has_keys = true;
    return HPERM_OK;
}

// Job order of the device queue. Ties keep the natural (expansion) order.
static std::vector<uint32_t> job_order(const hperm_jobs *j, int order, uint64_t seed) {
    const size_t nd = j->tab.desc.size();
    std::vector<uint32_t> ord(nd);
    std::iota(ord.begin(), ord.end(), 0u);
    auto key = [&](uint32_t k) { return j->has_keys ? j->keys[k] : 0.0f; };
    if (order == HPERM_ORDER_ESTIMATE) {
        // stable LSD radix sort on the keys, non-increasing: map each float to an unsigned
        // integer that increases with the float, then complement it
        std::vector<uint32_t> kb(nd), tmp(nd);
        for (size_t k = 0; k < nd; ++k) {
            uint32_t b;
            const float f = key((uint32_t)k);
            memcpy(&b, &f, 4);
            b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
            kb[k] = ~b;
        }
        std::vector<uint32_t> cnt(1 << 16);
        for (int pass = 0; pass < 2; ++pass) {
            const int shift = 16 * pass;
            std::fill(cnt.begin(), cnt.end(), 0u);
            for (uint32_t k : ord) cnt[(kb[k] >> shift) & 0xffff]++;
            uint32_t sum = 0;
            for (auto &c : cnt) {
                const uint32_t x = c;
                c = sum;
                sum += x;
            }
            for (uint32_t k : ord) tmp[cnt[(kb[k] >> shift) & 0xffff]++] = k;
            ord.swap(tmp);
        }
    } else if (order == HPERM_ORDER_EXACT_COST) {
        std::stable_sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) {
            const int ma = j->tab.desc[a].m, mb = j->tab.desc[b].m;
            if (ma != mb) return ma > mb;
            return key(a) > key(b);
        });
    } else if (order == HPERM_ORDER_RANDOM) {
        // Fisher-Yates driven by SplitMix64 outputs
        for (size_t i = nd; i > 1; --i) {
            uint64_t z = seed + (uint64_t)i * 0x9E3779B97F4A7C15ull;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            std::swap(ord[i - 1], ord[(size_t)(z % i)]);
        }
    }
    return ord;
}

// Lane chunk of a job for the one-launch-per-job comparator: the context's chunk_log2 when
// set, else about 256 waves per launch (one per four SIMDs) when the job is large enough.
static int plain_chunk(int m, int opt) {
    int c = opt > 0 ? opt : m - 1 - 6 - 8;
    if (c < 0) c = 0;
    if (c > 10 && opt <= 0) c = 10;
    if (c > 12) c = 12;
    if (c > m - 1) c = m - 1 > 0 ? m - 1 : 0;
    if (c < m - 32) c = m - 32;
    return c;
}

static uint64_t items_of(int m, int c) {
    const int e = m - 1 - 6 - c;
    return e > 0 ? (1ull << e) : 1ull;
}
uint64_t job_items(int m, int c) { return items_of(m, c); }

// Exact permanent of one job from its accumulator (see JobAcc). Returns false when an
// integrity check fails (2^(m-1) must divide V in the 2-adic rings, the value must be
// non-negative and within the proven bound).
static bool job_value(const JobDesc &d, const JobAcc &a, double log2_bound, U512 *out) {
    const int m = d.m;
    const int sh = m - 1;
    *out = U512();
    if (a.flag == HP_ACC_NORMALISED) {   // per(B) itself, as 32-bit limb sums
        for (int l = 3; l >= 0; --l) {
            U512 t;
            t.w[0] = a.l[l];
            for (int z = 0; z < l; ++z) t.mul_u64(1ull << 32);
            out->add(t);
        }
    } else if (d.arith == HP_W64 || d.arith == HP_W128) {
        i128 V;
        if (d.arith == HP_W64) {
            V = (int64_t)a.l[0];
        } else {
            u128 u = (u128)a.l[0] + ((u128)a.l[1] << 32) + ((u128)a.l[2] << 64) + ((u128)a.l[3] << 96);
            V = (i128)u;
        }
        if (sh & 1) V = -V;
        if (V < 0) return false;
        const u128 uv = (u128)V;
        if (sh > 0 && (uv & (((u128)1 << sh) - 1)) != 0) return false;
        out->add_u128(uv >> sh);
    } else {
        const uint64_t P[3] = {(1ull << 61) - HP_C0, (1ull << 61) - HP_C1, (1ull << 61) - HP_C2};
        uint64_t r[3];
        for (int k = 0; k < 3; ++k) {
            const u128 v = (u128)a.l[2 * k] + ((u128)a.l[2 * k + 1] << 32);
            uint64_t x = (uint64_t)(v % P[k]);
            // per = (-1)^(m-1) * (2^-1)^(m-1) * V (mod p)
            x = mulmod(x, powmod(invmod(2, P[k]), (uint64_t)sh, P[k]), P[k]);
            if ((sh & 1) && x) x = P[k] - x;
            r[k] = x;
        }
        // Garner: x = r0 + p0 * t1 + p0 p1 * t2
        const uint64_t t1 = mulmod((r[1] + P[1] - r[0] % P[1]) % P[1], invmod(P[0] % P[1], P[1]), P[1]);
        const uint64_t x01_mod_p2 = (uint64_t)(((u128)r[0] + (u128)P[0] % P[2] * t1) % P[2]);
        const uint64_t p01_mod_p2 = mulmod(P[0] % P[2], P[1] % P[2], P[2]);
        const uint64_t t2 = mulmod((r[2] + P[2] - x01_mod_p2) % P[2], invmod(p01_mod_p2, P[2]), P[2]);
        U512 x;
        x.w[0] = t2;
        x.mul_u64(P[1]);
        U512 y;
        y.w[0] = t1;
        x.add(y);
        x.mul_u64(P[0]);
        U512 z;
        z.w[0] = r[0];
        x.add(z);
        *out = x;
    }
    const int bits = out->bits();
    if (bits > (int)std::ceil(log2_bound) + 1) return false;
    return true;
}

// Algorithmic 32-bit VALU issue slots of one ring multiply by a 32-bit factor and of one
// ring addition. On gfx950 v_mad_u64_u32 and v_mul_lo_u32 issue at half the rate of simple
// 32-bit operations (2 slots), other 32-bit operations take 1 slot:
//   mod 2^64 : 64x32 product = v_mad_u64_u32 + v_mul_lo_u32 + add           -> 2 + 2 + 1 = 5
//              64-bit addition = add with carry out + add with carry in      -> 2
//   mod 2^128: 3 v_mad_u64_u32 + v_mul_lo_u32 + add                         -> 9; addition 4
//   residues : per prime a 61x24-bit product (2 multiplies), the fold by 2^61 = c (shift, mask,
//              multiply-add) and one conditional subtraction               -> 11; addition 3;
//              three primes
static double ring_mul_slots(int ring) { return ring == HP_W64 ? 5.0 : ring == HP_W128 ? 9.0 : 33.0; }
static double ring_add_slots(int ring) { return ring == HP_W64 ? 2.0 : ring == HP_W128 ? 4.0 : 9.0; }

// Algorithmic work of one job for the suffix-product Gray walk: every lane chunk of L = 2^c
// Gray indices starts with the product of all m row values (m ring multiplies); inside the
// chunk, column j < c flips L / 2^(j+1) times and each flip updates its nnz(j) row values and
// re-multiplies the hi[j] suffix products below the changed rows; every term is one ring
// addition. In the paired walk (variant v = 1, 2; b = v + 1 rows below the pair boundary) the
// L / 2 flips of column 0 give way to one pair sum each (two products of b rows and one
// multiply by the suffix above them: 2(b - 1) + 1 ring multiplies and one ring addition per
// pair), and the other flips re-multiply only from row b up. In the four-step walks (variant
// 6: column 0 on rows 0..1, column 1 on rows of 2..4, b = 5; variant 7: rows 0..2 and rows of
// 3..5, b = 6; row values below 2^7) the flips of columns 0 and 1 give way to one block sum
// per four steps: the products of A and of B without and with their column and the two
// differences in FP32 (2(a - 1) + 4 multiplies, a + 3 shifted rows, 2 differences: 13 / 16
// full-rate slots), two conversions and one 24-bit product of the differences (4 slots), the
// 64 x 64-bit multiply by the suffix (7 slots at the weights below: 1.4 ring multiplies) and
// one ring addition. The other flips re-multiply only from row b up. `extra` holds the
// full-rate slots that are neither ring operations nor row updates.
struct JobWork {
    double mults, adds, updates;
    double extra = 0.0;
};
static JobWork job_work(const JobDesc &d, const uint32_t *data, int chunk, int variant) {
    const int m = d.m;
    const uint32_t *cs = data + hp_data_index(d) + m;
    const uint32_t *hi = cs + m;
    const double L = std::ldexp(1.0, chunk);
    const double chunks = std::ldexp(1.0, m - 1) / L;
    double mults = m, updates = 0, adds = L;
    if (variant >= 6) {
        const double b = variant == 6 ? 5.0 : 6.0;   // the kernel's boundary row
        const double blocks = L / 4;
        mults += blocks * 1.4;
        const double extra = blocks * (variant == 6 ? 17.0 : 20.0);
        for (int j = 2; j < chunk && j + 1 < m; ++j) {
            const double flips = L / std::ldexp(1.0, j + 1);
            updates += flips * (cs[j + 1] - cs[j]);
            mults += flips * std::max(0.0, (double)hi[j] - b);
        }
        return {chunks * mults, chunks * blocks, chunks * updates, chunks * extra};
    }
    for (int j = 0; j < chunk && j + 1 < m; ++j) {
        const double flips = L / std::ldexp(1.0, j + 1);
        updates += flips * (cs[j + 1] - cs[j]);
        if (variant > 0) {
            const double b = variant + 1;
            mults += j == 0 ? flips * (2.0 * (b - 1.0) + 1.0) : flips * std::max(0.0, (double)hi[j] - b);
        } else {
            mults += flips * hi[j];
        }
    }
    if (variant > 0) adds = L / 2;
    return {chunks * mults, chunks * adds, chunks * updates};
}

// The integer x in [0, p0 p1 p2) with x = (res[2k] + 2^32 res[2k+1]) mod p_k (Garner).
static U512 crt3(const unsigned long long *res) {
    const uint64_t P[3] = {(1ull << 61) - HP_C0, (1ull << 61) - HP_C1, (1ull << 61) - HP_C2};
    uint64_t r[3];
    for (int k = 0; k < 3; ++k) r[k] = (uint64_t)(((u128)res[2 * k] + ((u128)res[2 * k + 1] << 32)) % P[k]);
    const uint64_t t1 = mulmod((r[1] + P[1] - r[0] % P[1]) % P[1], invmod(P[0] % P[1], P[1]), P[1]);
    const uint64_t x01 = (uint64_t)(((u128)r[0] + (u128)(P[0] % P[2]) * t1) % P[2]);
    const uint64_t p01 = mulmod(P[0] % P[2], P[1] % P[2], P[2]);
    const uint64_t t2 = mulmod((r[2] + P[2] - x01) % P[2], invmod(p01, P[2]), P[2]);
    U512 x;
    x.w[0] = t2;
    x.mul_u64(P[1]);
    U512 y;
    y.w[0] = t1;
    x.add(y);
    x.mul_u64(P[0]);
    U512 z;
    z.w[0] = r[0];
    x.add(z);
    return x;
}

// per(A) of a problem from its device accumulator: the 32-bit limb sums of its 2-adic-ring
// jobs plus the CRT of its residue sums.
U512 prob_value(const ProbAcc &q) {
    U512 v;
    for (int l = 3; l >= 0; --l) {   // sum_l lim[l] 2^(32 l)
        U512 t;
        t.w[0] = q.lim[l];
        for (int z = 0; z < l; ++z) t.mul_u64(1ull << 32);
        v.add(t);
    }
    bool any_res = false;
    for (int z = 0; z < 6; ++z) any_res |= q.res[z] != 0;
    if (any_res) v.add(crt3(q.res));
    return v;
}

void fill_result(const U512 &v, hperm_result *r) {
    for (int k = 0; k < 8; ++k) r->limb[k] = v.w[k];
    r->nlimb = v.nlimb();
}

static hperm_status ensure_launch_events(Dev *c, size_t pairs) {
    while (c->launch_ev.size() < 2 * pairs) {
        hipEvent_t e;
        hperm_status s = hip_check(c, hipEventCreate(&e), "hipEventCreate");
        if (s) return s;
        c->launch_ev.push_back(e);
    }
    return HPERM_OK;
}

// The persistent queue's launch groups of a job table (independent of the job order): group
// g = (order bucket, ring, walk variant) from the largest bucket and the widest ring down. The
// order-20 bucket exists for the many jobs of the default cut-off; when a (ring, walk) group of
// it is small, its jobs join the order-24 group instead (whose kernel takes them too), saving
// a launch and its drain tail. With split_order t > 0 the mod-2^64 jobs of order t+1..24 form
// one more group, last, for the device continuation of H_per (variant 3, one item per job).
static constexpr int kSplitVariant = 3;
static bool split_eligible(const JobDesc &d, int split) {
    return split > 0 && d.arith == HP_W64 && d.m > split && d.m <= HP_SPLIT_MAX_M;
}
// The split order in effect: the device continuation follows H_per's rule only for s_leaf <= 5
// (its nodes have at most two children).
int split_in_effect(const hperm_opts &o) { return o.s_leaf <= 5 ? o.split_order : 0; }
uint64_t split_wide_total(const std::vector<JobDesc> &desc, const hperm_opts &o) {
    const int split = split_in_effect(o);
    uint64_t w = 0;
    for (const JobDesc &d : desc)
        if (split_eligible(d, split)) w += split_wide_entries(d.m);
    return w;
}

static void build_queue_groups(hperm_jobs *j, int split) {
    const std::vector<JobDesc> &dsc = j->tab.desc;
    const size_t nd = dsc.size();
    constexpr int NV = 5;   // walks 0, 1, 2 and the four-step walks (variants 6, 7) at indices 3, 4
    auto vindex = [](int v) { return v >= 6 ? v - 3 : v; };
    auto vof = [](int i) { return i >= 3 ? i + 3 : i; };
    constexpr int NG = HP_RNW_BUCKETS * HP_NRING * NV;
    constexpr int SPLIT_G = NG;   // the device H_per group
    constexpr uint64_t kSmallGroupItems = 16384;
    std::vector<uint8_t> raw(nd);
    j->qitems.resize(nd);
    uint64_t items_raw[NG + 1] = {0};
    for (size_t k = 0; k < nd; ++k) {
        const JobDesc &d = dsc[k];
        int g;
        if (split_eligible(d, split)) {
            g = SPLIT_G;
            j->qitems[k] = 1;
        } else {
            g = ((HP_RNW_BUCKETS - 1 - bucket_of(d.m)) * HP_NRING + (HP_NRING - 1 - d.arith)) * NV +
                vindex(walk_variant(d, d.chunk_log2));
            j->qitems[k] = items_of(d.m, d.chunk_log2);
        }
        raw[k] = (uint8_t)g;
        items_raw[g] += j->qitems[k];
    }
    int remap[NG + 1];
    for (int g = 0; g < NG; ++g) {
        const int bucket = HP_RNW_BUCKETS - 1 - g / (NV * HP_NRING);
        remap[g] = (bucket == 1 && items_raw[g] < kSmallGroupItems) ? g - NV * HP_NRING : g;
    }
    remap[SPLIT_G] = SPLIT_G;
    hperm_jobs::QueueGroup acc[NG + 1];
    for (int g = 0; g < NG; ++g)
        acc[g] = hperm_jobs::QueueGroup{HP_NRING - 1 - (g / NV) % HP_NRING, HP_RNW_BUCKETS - 1 - g / (NV * HP_NRING),
                                        vof(g % NV), 0, 0, 0, 0.0, 0.0, 0.0};
    acc[SPLIT_G] = hperm_jobs::QueueGroup{HP_W64, bucket_of(HP_SPLIT_MAX_M), kSplitVariant, 0, 0, 0, 0.0, 0.0, 0.0};
    for (size_t k = 0; k < nd; ++k) {
        const JobDesc &d = dsc[k];
        hperm_jobs::QueueGroup &q = acc[remap[raw[k]]];
        q.n++;
        q.items += j->qitems[k];
        q.terms += 1ull << (d.m - 1);
        if (raw[k] == SPLIT_G) {   // its work is known only after the run
            q.mmax = std::max(q.mmax, (int)d.m);
            q.wide += split_wide_entries(d.m);
            continue;
        }
        const JobWork wk = job_work(d, j->tab.data.data(), d.chunk_log2, walk_variant(d, d.chunk_log2));
        q.mults += wk.mults;
        q.adds += wk.adds;
        q.updates += wk.updates;
        q.extra += wk.extra;
    }
    int index[NG + 1];
    j->qgroups.clear();
    for (int g = 0; g <= NG; ++g) {
        index[g] = (int)j->qgroups.size();
        if (acc[g].n) j->qgroups.push_back(acc[g]);
    }
    j->qgroup.resize(nd);
    for (size_t k = 0; k < nd; ++k) j->qgroup[k] = (uint8_t)index[remap[raw[k]]];
    j->qsplit = split;
}

// The lane chunk of a job under a tuning offset (the limits of the expansion's own choice:
// at most 12, at most m - 1, at least m - 32).
static int tuned_chunk(int m, int c0, int delta, int cmin) {
    int c = c0 + delta;
    if (c > 12) c = 12;
    if (c > m - 1) c = std::max(0, m - 1);
    if (c < cmin) c = std::min(cmin, std::max(0, m - 1));
    if (c < m - 32) c = m - 32;
    return c;
}

// Brings the job table's lane chunks in line with the context's tuning table (each job's own
// chunk plus its group's offset; the expansion's chunks when untuned).
static void apply_tuning(Dev *c, hperm_jobs *j) {
    const size_t nd = j->tab.desc.size();
    TuneTable *tt = c->tune.get();
    uint64_t ver = 0;
    std::map<int, TuneEntry> table;
    if (tt) {
        std::lock_guard<std::mutex> lk(tt->mu);
        ver = tt->version;
        table = tt->e;
    }
    if (j->tune_table == (const void *)tt && j->tune_version == ver) return;
    if (j->chunk0.size() != nd) {
        j->chunk0.resize(nd);
        for (size_t k = 0; k < nd; ++k) j->chunk0[k] = j->tab.desc[k].chunk_log2;
    }
    bool changed = false;
    for (size_t k = 0; k < nd; ++k) {
        JobDesc &d = j->tab.desc[k];
        JobDesc d0 = d;
        d0.chunk_log2 = j->chunk0[k];
        int want = d0.chunk_log2;
        const int v0 = walk_variant(d0, d0.chunk_log2);
        const auto it = table.find(tune_key(d.arith, bucket_of(d.m), v0));
        if (it != table.end() && d0.chunk_log2 > 0)
            want = tuned_chunk(d.m, d0.chunk_log2, it->second.chunk_delta, v0 >= 6 ? 2 : 1);
        if (d.chunk_log2 != want) {
            d.chunk_log2 = (uint8_t)want;
            changed = true;
        }
    }
    if (changed) {   // new chunks: new work items and groups, and the descriptors go up again
        j->qgroup.clear();
        if (c->resident_jobs == j->id) c->resident_jobs = 0;
    }
    j->tune_table = tt;
    j->tune_version = ver;
}

// The persistent grid of a launch group under the tuning table (0: the resident grid).
static int tuned_grid(Dev *c, int ring, int bucket, int variant) {
    if (!c->tune) return 0;
    std::lock_guard<std::mutex> lk(c->tune->mu);
    const auto it = c->tune->e.find(tune_key(ring, bucket, variant));
    if (it == c->tune->e.end() || it->second.grid_pct == 100) return 0;
    int full = 0;
    if (persistent_grid(ring, bucket, variant, &full) != hipSuccess) return 0;
    return std::max(1, full * it->second.grid_pct / 100);
}

static hperm_status ensure_host_prob(Dev *c, size_t np) {
    if (c->host_prob_cap >= np && c->host_split) return HPERM_OK;
    if (c->host_prob_cap < np) {
        if (c->host_prob) (void)hipHostFree(c->host_prob);
        c->host_prob = nullptr;
        c->host_prob_cap = 0;
        hperm_status s = hip_check(c, hipHostMalloc((void **)&c->host_prob, std::max<size_t>(np, 1) * sizeof(ProbAcc),
                                                    hipHostMallocDefault), "hipHostMalloc");
        if (s) return s;
        c->host_prob_cap = std::max<size_t>(np, 1);
    }
    if (!c->host_split)
        return hip_check(c, hipHostMalloc((void **)&c->host_split, HP_SPLIT_STATS * sizeof(unsigned long long),
                                          hipHostMallocDefault), "hipHostMalloc");
    return HPERM_OK;
}

// Step 4 and the downloads after the launches: per-job accumulators, or the per-problem sums
// of the recombination (into pinned host memory).
static hperm_status enqueue_results(Dev *c, hperm_jobs *j, JobAcc *accs, bool want_per_job) {
    const size_t nd = j->tab.desc.size();
    const int np = j->tab.n_problems;
    hperm_status s;
    if (c->split_launch >= 0) {
        s = hip_check(c, hipMemcpyAsync(c->host_split, c->buf[B_SPLIT].ptr, HP_SPLIT_STATS * sizeof(unsigned long long),
                                        hipMemcpyDeviceToHost, c->stream), "download split counters");
        if (s) return s;
    }
    if (want_per_job) {
        c->host_acc.resize(nd);
        return hip_check(c, hipMemcpyAsync(c->host_acc.data(), accs, nd * sizeof(JobAcc),
                                           hipMemcpyDeviceToHost, c->stream), "download job values");
    }
    ProbAcc *pd = (ProbAcc *)c->buf[B_PROB].ptr;
    s = hip_check(c, launch_fill_u64((unsigned long long *)pd, (uint64_t)np * (sizeof(ProbAcc) / 8), 0ull,
                                     c->stream), "clear problem accumulators");
    if (s) return s;
    s = hip_check(c, launch_recombine((const JobDesc *)c->buf[B_DESC].ptr, accs, (uint32_t)nd, pd, c->stream),
                  "recombine launch");
    if (s) return s;
    return hip_check(c, hipMemcpyAsync(c->host_prob, pd, np * sizeof(ProbAcc), hipMemcpyDeviceToHost,
                                       c->stream), "download problem values");
}

// The device operations of a persistent run after the queue upload: clears, the launches of
// the groups (with an event pair around each when `events`), Step 4 and the downloads. Only
// stream work (kernels and copies between device and pinned memory): capturable in a graph.
static hperm_status enqueue_persistent_ops(Dev *c, hperm_jobs *j, const JobDesc *d_desc, const uint32_t *d_data,
                                           const std::vector<size_t> &goff, bool events, bool want_per_job) {
    const size_t nd = j->tab.desc.size();
    JobAcc *accs = (JobAcc *)c->buf[B_ACCS].ptr;
    unsigned long long *head = (unsigned long long *)c->buf[B_HEAD].ptr;
    hperm_status s = hip_check(c, launch_fill_u64((unsigned long long *)accs, nd * (sizeof(JobAcc) / 8), 0ull,
                                                  c->stream), "clear accumulators");
    if (s) return s;
    s = hip_check(c, launch_fill_u64(head, 64, 0ull, c->stream), "clear queue heads");
    if (s) return s;
    // per-job work cycles (opt-in): cleared here, downloaded by run_finish
    unsigned long long *cyc = nullptr;
    if (c->timed) {
        cyc = (unsigned long long *)c->buf[B_CYCLES].ptr;
        s = hip_check(c, launch_fill_u64(cyc, nd, 0ull, c->stream), "clear job cycles");
        if (s) return s;
    }
    if (events) {
        s = hip_check(c, hipEventRecord(c->ev0, c->stream), "event");
        if (s) return s;
    }
    for (size_t gi = 0; gi < j->qgroups.size(); ++gi) {
        const hperm_jobs::QueueGroup &g = j->qgroups[gi];
        if (g.variant == kSplitVariant) {
            s = hip_check(c, launch_fill_u64((unsigned long long *)c->buf[B_SPLIT].ptr, HP_SPLIT_STATS, 0ull, c->stream),
                          "clear split counters");
            if (s) return s;
        }
        if (events) {
            s = hip_check(c, hipEventRecord(c->launch_ev[2 * gi], c->stream), "event");
            if (s) return s;
        }
        if (g.variant == kSplitVariant)
            s = hip_check(c, launch_split_jobs(d_desc, d_data, (const float *)c->buf[B_BOUND].ptr,
                                               (const uint32_t *)c->buf[B_QUEUE].ptr + goff[gi], (uint32_t)g.n,
                                               (uint32_t)nd, split_in_effect(c->opts), g.mmax, c->opts.s_leaf,
                                               head + gi, accs, (unsigned long long *)c->buf[B_SPLIT].ptr,
                                               c->buf[B_SPLIT_WIDE].ptr, split_wide_capacity(g.wide, g.n), cyc,
                                               c->stream),
                          "device H_per launch");
        else
            s = hip_check(c, launch_rnw_persistent(g.ring, g.bucket, g.variant, d_desc, d_data,
                                                   (const uint32_t *)c->buf[B_QUEUE].ptr + goff[gi],
                                                   (const uint64_t *)c->buf[B_ITEMS].ptr + goff[gi],
                                                   (uint32_t)g.n, g.items, head + gi, accs, cyc,
                                                   tuned_grid(c, g.ring, g.bucket, g.variant), c->stream),
                          "rnw_persistent launch");
        if (s) return s;
        if (events) {
            s = hip_check(c, hipEventRecord(c->launch_ev[2 * gi + 1], c->stream), "event");
            if (s) return s;
        }
    }
    if (events) {
        s = hip_check(c, hipEventRecord(c->ev1, c->stream), "event");
        if (s) return s;
    }
    return enqueue_results(c, j, accs, want_per_job);
}

// What a captured graph depends on: the job table, the device buffers, the launch groups and the
// options the launches take.
static GraphKey graph_key(Dev *c, hperm_jobs *j) {
    GraphKey k;
    k.jobs_id = j->id;
    k.nd = j->tab.desc.size();
    k.np = j->tab.n_problems;
    for (int b = 0; b < B_COUNT; ++b) k.bufs[b] = c->buf[b].ptr;
    k.split = split_in_effect(c->opts);
    k.s_leaf = c->opts.s_leaf;
    k.host_prob = c->host_prob;
    k.host_split = c->host_split;
    k.tune_table = c->tune.get();
    k.tune_version = c->tune ? c->tune->version : 0;
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](uint64_t x) { h = (h ^ x) * 1099511628211ull; };
    for (const auto &g : j->qgroups) {
        mix((uint64_t)g.ring);
        mix((uint64_t)g.bucket);
        mix((uint64_t)g.variant);
        mix(g.n);
        mix(g.items);
        mix((uint64_t)g.mmax);
        mix(g.wide);
    }
    k.groups = h;
    return k;
}

hperm_status run_enqueue(Dev *c, hperm_jobs *j, int order, int persistent, bool want_per_job) {
    const size_t nd = j->tab.desc.size();
    const int np = j->tab.n_problems;
    if (order < 0 || order > 3) return set_error(c, HPERM_E_INVALID, "unknown order");
    if ((order == HPERM_ORDER_ESTIMATE) && !j->has_keys && nd)
        return set_error(c, HPERM_E_INVALID, "ORDER_ESTIMATE needs hperm_estimate first");
    c->want_per_job = want_per_job;
    c->persistent = persistent != 0;
    c->graphed = false;
    c->launches.clear();
    if (!nd) return HPERM_OK;
    hperm_status s;
    if (!c->ev0) {
        s = hip_check(c, hipEventCreate(&c->ev0), "hipEventCreate");
        if (s) return s;
        s = hip_check(c, hipEventCreate(&c->ev1), "hipEventCreate");
        if (s) return s;
    }
    // per-mode chunk sizes: the persistent queue uses the jobs' own chunks
    std::vector<JobDesc> &desc_plain = c->h_desc_plain;
    if (!persistent) {
        desc_plain = j->tab.desc;
        for (auto &d : desc_plain) d.chunk_log2 = (uint8_t)plain_chunk(d.m, c->opts.chunk_log2);
    }
    // the persistent queue: the launch groups (cached per job table), each group's jobs in
    // the chosen order, and inclusive prefix sums of their work items
    std::vector<uint32_t> &queue = c->h_queue;
    std::vector<uint64_t> &item_end = c->h_items;
    std::vector<size_t> goff;
    if (persistent) {
        const int split = split_in_effect(c->opts);
        apply_tuning(c, j);
        if (j->qgroup.size() != nd || j->qsplit != split) build_queue_groups(j, split);
        const std::vector<uint32_t> ord = job_order(j, order, c->opts.seed);
        const size_t ng = j->qgroups.size();
        goff.assign(ng + 1, 0);
        for (size_t g = 0; g < ng; ++g) goff[g + 1] = goff[g] + j->qgroups[g].n;
        std::vector<size_t> pos(goff.begin(), goff.end() - 1);
        queue.resize(nd);
        item_end.resize(nd);
        for (uint32_t k : ord) queue[pos[j->qgroup[k]]++] = k;
        for (size_t g = 0; g < ng; ++g) {
            uint64_t acc = 0;
            for (size_t q = goff[g]; q < goff[g + 1]; ++q) item_end[q] = acc += j->qitems[queue[q]];
        }
    }
    s = upload_jobs(c, j);
    if (s) return s;
    if (persistent) {
        s = ensure_buf(c, B_QUEUE, nd * sizeof(uint32_t));
        if (s) return s;
        s = ensure_buf(c, B_ITEMS, nd * sizeof(uint64_t));
        if (s) return s;
    }
    s = ensure_buf(c, B_ACCS, nd * sizeof(JobAcc));
    if (s) return s;
    s = ensure_buf(c, B_HEAD, 64 * sizeof(unsigned long long));
    if (s) return s;
    s = ensure_buf(c, B_PROB, (size_t)np * sizeof(ProbAcc));
    if (s) return s;
    if (!persistent) {
        s = ensure_buf(c, B_DESC_PLAIN, nd * sizeof(JobDesc));
        if (s) return s;
    }
    c->timed = persistent && c->opts.time_jobs != 0;
    c->split_launch = -1;
    if (persistent && split_in_effect(c->opts)) {
        s = ensure_buf(c, B_SPLIT, HP_SPLIT_STATS * sizeof(unsigned long long));
        if (s) return s;
        const hperm_jobs::QueueGroup &last = j->qgroups.back();
        s = ensure_buf(c, B_SPLIT_WIDE,
                       split_wide_bytes(last.variant == kSplitVariant ? split_wide_capacity(last.wide, last.n) : 0));
        if (s) return s;
    }
    if (c->timed) {
        s = ensure_buf(c, B_CYCLES, nd * sizeof(unsigned long long));
        if (s) return s;
    }
    if (c->resident_jobs != j->id) {   // an arena re-layout moved the job table: upload again
        s = upload_jobs(c, j);
        if (s) return s;
    }
    const JobDesc *d_desc = (const JobDesc *)c->buf[B_DESC].ptr;
    if (!persistent) {
        s = hip_check(c, hipMemcpyAsync(c->buf[B_DESC_PLAIN].ptr, desc_plain.data(),
                                        nd * sizeof(JobDesc), hipMemcpyHostToDevice, c->stream),
                      "upload plain descriptors");
        if (s) return s;
        d_desc = (const JobDesc *)c->buf[B_DESC_PLAIN].ptr;
    }
    if (persistent) {
        s = hip_check(c, hipMemcpyAsync(c->buf[B_QUEUE].ptr, queue.data(), nd * 4,
                                        hipMemcpyHostToDevice, c->stream), "upload queue");
        if (s) return s;
        s = hip_check(c, hipMemcpyAsync(c->buf[B_ITEMS].ptr, item_end.data(), nd * 8,
                                        hipMemcpyHostToDevice, c->stream), "upload item ends");
        if (s) return s;
    }
    JobAcc *accs = (JobAcc *)c->buf[B_ACCS].ptr;
    const uint32_t *d_data = (const uint32_t *)c->buf[B_DATA].ptr;
    s = ensure_host_prob(c, (size_t)np);   // Step 4's staging and the split counters, pinned
    if (s) return s;
    if (persistent) {
        c->launches.clear();
        for (size_t gi = 0; gi < j->qgroups.size(); ++gi) {
            const hperm_jobs::QueueGroup &g = j->qgroups[gi];
            hperm_launch_stat st{};
            st.ring = g.ring;
            st.bucket = g.bucket;
            st.n_jobs = (int32_t)g.n;
            st.persistent = 1;
            st.variant = g.variant;
            st.items = g.items;
            st.terms = g.terms;
            st.row_updates = (uint64_t)g.updates;
            st.alg_slots = g.mults * ring_mul_slots(g.ring) + g.adds * ring_add_slots(g.ring) + g.updates + g.extra;
            if (g.variant == kSplitVariant) {
                c->split_launch = (int)gi;
                st.reserved = split_grid(split_in_effect(c->opts), g.mmax);   // its resident waves
            }
            c->launches.push_back(st);
        }
        const bool graph = c->opts.use_graphs != 0 && !want_per_job && !c->timed;
        c->graphed = graph;
        if (!graph) {
            s = ensure_launch_events(c, j->qgroups.size());
            if (s) return s;
            return enqueue_persistent_ops(c, j, d_desc, d_data, goff, true, want_per_job);
        }
        // the device part as a HIP graph: captured once per job table, buffers, launch groups
        // and tuning, replayed afterwards (the queue upload above stays outside the graph)
        GraphKey key = graph_key(c, j);
        if (!c->graph_exec || !(c->graph_key == key)) {
            if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
            c->graph_exec = nullptr;
            s = hip_check(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
            if (s) return s;
            const hperm_status s_ops = enqueue_persistent_ops(c, j, d_desc, d_data, goff, false, false);
            hipGraph_t gr = nullptr;
            const hipError_t e_end = hipStreamEndCapture(c->stream, &gr);
            if (s_ops) {
                if (gr) (void)hipGraphDestroy(gr);
                return s_ops;
            }
            s = hip_check(c, e_end, "hipStreamEndCapture");
            if (s) return s;
            s = hip_check(c, hipGraphInstantiate(&c->graph_exec, gr, nullptr, nullptr, 0), "hipGraphInstantiate");
            (void)hipGraphDestroy(gr);
            if (s) return s;
            c->graph_key = key;
            c->graph_captures++;
        }
        s = hip_check(c, hipEventRecord(c->ev0, c->stream), "event");
        if (s) return s;
        s = hip_check(c, hipGraphLaunch(c->graph_exec, c->stream), "hipGraphLaunch");
        if (s) return s;
        return hip_check(c, hipEventRecord(c->ev1, c->stream), "event");
    }
    unsigned long long *head = (unsigned long long *)c->buf[B_HEAD].ptr;
    s = hip_check(c, launch_fill_u64((unsigned long long *)accs, nd * (sizeof(JobAcc) / 8), 0ull,
                                     c->stream), "clear accumulators");
    if (s) return s;
    s = hip_check(c, launch_fill_u64(head, 64, 0ull, c->stream), "clear queue heads");
    if (s) return s;
    s = hip_check(c, hipEventRecord(c->ev0, c->stream), "event");
    if (s) return s;
    // one launch per job, natural order
    for (size_t k = 0; k < nd; ++k) {
        const JobDesc &d = desc_plain[k];
        const int v = walk_variant(d, d.chunk_log2);
        s = hip_check(c, launch_rnw_single(d.arith, bucket_of(d.m), v, d_desc, d_data, (uint32_t)k,
                                           items_of(d.m, d.chunk_log2), accs, c->stream),
                      "rnw_single launch");
        if (s) return s;
    }
    hperm_launch_stat st{};
    st.ring = -1;
    st.bucket = -1;
    st.n_jobs = (int32_t)nd;
    for (size_t k = 0; k < nd; ++k) {
        const JobDesc &d = desc_plain[k];
        const uint64_t t = 1ull << (d.m - 1);
        const JobWork wk = job_work(d, j->tab.data.data(), d.chunk_log2, walk_variant(d, d.chunk_log2));
        st.items += items_of(d.m, d.chunk_log2);
        st.terms += t;
        st.row_updates += (uint64_t)wk.updates;
        st.alg_slots += wk.mults * ring_mul_slots(d.arith) + wk.adds * ring_add_slots(d.arith) + wk.updates + wk.extra;
    }
    c->launches.push_back(st);   // all single launches as one record (ms = whole span)
    s = hip_check(c, hipEventRecord(c->ev1, c->stream), "event");
    if (s) return s;
    return enqueue_results(c, j, accs, want_per_job);
}

hperm_status run_finish(Dev *c, hperm_jobs *j, hperm_result *per_job, hperm_result *totals,
                        double *t_rnw) {
    const size_t nd = j->tab.desc.size();
    const int np = j->tab.n_problems;
    std::vector<U512> sums(np);
    std::vector<int> nj(np, 0), maxm(np, 0), amask(np, 0);
    std::vector<uint64_t> terms(np, 0);
    *t_rnw = 0.0;
    if (nd) {
        hperm_status s = hip_check(c, hipStreamSynchronize(c->stream), "R-NW");
        if (s) return s;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
        *t_rnw = ms * 1e-3;
        if (c->persistent) {
            for (size_t gi = 0; gi < c->launches.size(); ++gi) {
                float lm = 0.0f;   // a replayed graph has no per-launch events: the whole span
                if (c->graphed) lm = gi == 0 ? ms : 0.0f;
                else (void)hipEventElapsedTime(&lm, c->launch_ev[2 * gi], c->launch_ev[2 * gi + 1]);
                c->launches[gi].ms = lm;
            }
            if (c->split_launch >= 0) {
                const unsigned long long *ss = c->host_split;
                hperm_launch_stat &st = c->launches[(size_t)c->split_launch];
                st.leaves = ss[0];
                st.leaf_terms = ss[1];
                st.splits = ss[2];
                st.split_stops = ss[3];
                st.deferred = ss[4];
                st.deferred_bound = ss[7];
                if (ss[5]) return set_error(c, HPERM_E_INTERNAL, "device H_per: leaf records lost");
                if (ss[6]) return set_error(c, HPERM_E_INTERNAL, "device H_per: a leaf value failed its integrity check");
            }
        } else if (!c->launches.empty()) {
            c->launches[0].ms = ms;
        }
        if (c->timed) {
            j->cycles.resize(nd);
            s = hip_check(c, hipMemcpy(j->cycles.data(), c->buf[B_CYCLES].ptr, nd * sizeof(uint64_t),
                                       hipMemcpyDeviceToHost), "download job cycles");
            if (s) return s;
            j->has_cycles = true;
        }
        for (size_t k = 0; k < nd; ++k) {
            const JobDesc &d = j->tab.desc[k];
            const int p = (int)d.problem;
            nj[p]++;
            maxm[p] = std::max(maxm[p], (int)d.m);
            amask[p] |= 1 << (d.arith + 1);
            terms[p] += 1ull << (d.m - 1);
        }
        if (c->want_per_job) {
            for (size_t k = 0; k < nd; ++k) {
                const JobDesc &d = j->tab.desc[k];
                U512 v;
                if (!job_value(d, c->host_acc[k], j->tab.log2_bound[k], &v))
                    return set_error(c, HPERM_E_INTERNAL, "a job value failed its integrity check (job " +
                                                              std::to_string(k) + ")");
                sums[d.problem].add(v);
                if (per_job) {
                    memset(&per_job[k], 0, sizeof(hperm_result));
                    fill_result(v, &per_job[k]);
                    per_job[k].n_jobs = 1;
                    per_job[k].max_m = d.m;
                    per_job[k].arith_mask = 1 << (d.arith + 1);
                    per_job[k].subset_terms = 1ull << (d.m - 1);
                }
            }
        } else {
            for (int p = 0; p < np; ++p) {
                const ProbAcc &q = c->host_prob[p];
                if (q.err)
                    return set_error(c, HPERM_E_INTERNAL, "a job value of problem " + std::to_string(p) +
                                                              " failed its integrity check");
                sums[p] = prob_value(q);
            }
        }
        for (int p = 0; p < np; ++p)
            if (!j->tab.direct_valid[p] && sums[p].bits() > (int)std::ceil(j->tab.problem_log2_bound[p]) + 1)
                return set_error(c, HPERM_E_INTERNAL, "a result exceeds its proven bound (problem " +
                                                          std::to_string(p) + ")");
    }
    for (int p = 0; p < np; ++p) {
        hperm_result &r = totals[p];
        memset(&r, 0, sizeof(r));
        U512 v = sums[p];
        if (j->tab.direct_valid[p]) {
            v = U512();
            v.w[0] = j->tab.direct_value[p];
        }
        fill_result(v, &r);
        r.n_jobs = nj[p];
        r.max_m = maxm[p];
        r.arith_mask = amask[p];
        r.subset_terms = terms[p];
        r.t_rnw_s = *t_rnw;
    }
    return HPERM_OK;
}

hperm_status run_jobs(Dev *c, hperm_jobs *j, int order, int persistent, hperm_result *per_job,
                      hperm_result *totals, double *t_rnw) {
    hperm_status s = run_enqueue(c, j, order, persistent, per_job != nullptr);
    if (s) return s;
    return run_finish(c, j, per_job, totals, t_rnw);
}

void dev_release(Dev *d) {
    if (d->stream) (void)hipStreamSynchronize(d->stream);
    for (auto &b : d->buf) {
        if (b.ptr && b.owned) (void)hipFree(b.ptr);
        b = DevBuf();
    }
    for (hipEvent_t e : d->launch_ev) (void)hipEventDestroy(e);
    d->launch_ev.clear();
    if (d->ev0) (void)hipEventDestroy(d->ev0);
    if (d->ev1) (void)hipEventDestroy(d->ev1);
    d->ev0 = d->ev1 = nullptr;
    if (d->host_prob) (void)hipHostFree(d->host_prob);
    d->host_prob = nullptr;
    d->host_prob_cap = 0;
    if (d->host_split) (void)hipHostFree(d->host_split);
    d->host_split = nullptr;
    if (d->graph_exec) (void)hipGraphExecDestroy(d->graph_exec);
    d->graph_exec = nullptr;
    d->resident_jobs = 0;
    d->resident_list = 0;
}

// The job order of the device expansion in effect: device_expand when it exceeds the split
// order in effect, else 0 (off).
int device_in_effect(const hperm_opts &o) {
    const int t = split_in_effect(o);
    return (t > 0 && o.device_expand > t) ? o.device_expand : 0;
}

// Problems the residue evaluation can take when the exact paths refuse them (an entry or a
// bound out of their range): order above the device expansion's, within its nodes.
bool residue_path(const hperm_opts &o, int n) {
    const int T = device_in_effect(o);
    return T > 0 && n > T && n <= HP_MAX_N;
}

// Problems the device expansion takes: order above T and a proven bound below 2^102.
bool device_path(const hperm_opts &o, const CsrView &v) {
    const int T = device_in_effect(o);
    if (T <= 0 || v.n <= T) return false;
    std::vector<uint32_t> root;
    double lb = 0.0;
    const int rc = pack_root_node(v, &root, &lb);
    return rc == 0 && lb <= 102.0;
}

}  // namespace hp

// ====================================================================== C ABI
extern "C" {

hperm_status hperm_version(int32_t *major, int32_t *minor) {
    if (!major || !minor) return HPERM_E_INVALID;
    *major = 1;
    *minor = 0;
    return HPERM_OK;
}

hperm_status hperm_default_opts(hperm_opts *o) {
    if (!o) return HPERM_E_INVALID;
    memset(o, 0, sizeof(*o));
    o->m_cut = 20;
    o->m_cap = 36;
    o->s_leaf = 5;
    o->arith = HPERM_ARITH_AUTO;
    o->order = HPERM_ORDER_ESTIMATE;
    o->trials = 32;
    o->seed = 1;
    o->chunk_log2 = 0;
    o->persistent = 1;
    o->host_threads = 0;
    o->split_order = 12;
    o->device_expand = 22;
    o->device_expand_mib = 0;
    return HPERM_OK;
}

static const char *check_opts(const hperm_opts *o) {
    if (o->m_cut < 1 || o->m_cut > HP_MAX_M) return "m_cut must be in [1, 40]";
    if (o->m_cap < o->m_cut || o->m_cap > HP_MAX_M) return "m_cap must be in [m_cut, 40]";
    if (o->s_leaf < 1) return "s_leaf must be >= 1";
    if (o->arith < 0 || o->arith > 3) return "unknown arith";
    if (o->order < 0 || o->order > 3) return "unknown order";
    if (o->trials < 1 || o->trials > 4096) return "trials must be in [1, 4096]";
    if (o->chunk_log2 < 0 || o->chunk_log2 > 12) return "chunk_log2 must be in [0, 12]";
    if (o->host_threads < 0 || o->host_threads > 64) return "host_threads must be in [0, 64]";
    if (o->max_table_mib < 0) return "max_table_mib must be >= 0";
    if (o->time_jobs != 0 && o->time_jobs != 1) return "time_jobs must be 0 or 1";
    if (o->use_graphs != 0 && o->use_graphs != 1) return "use_graphs must be 0 or 1";
    if (o->serve_limit_ms < 0) return "serve_limit_ms must be >= 0";
    if (o->split_order != 0 && (o->split_order < HP_SPLIT_MIN_T || o->split_order >= HP_SPLIT_MAX_M))
        return "split_order must be 0 or in [7, 23]";
    if (o->device_expand < 0 || o->device_expand > HP_SPLIT_MAX_M) return "device_expand must be in [0, 24]";
    if (o->device_expand_mib < 0) return "device_expand_mib must be >= 0";
    return nullptr;
}

hperm_status hperm_ctx_create(const hperm_opts *opts, void *stream, hperm_ctx **out) {
    if (!out) return HPERM_E_INVALID;
    *out = nullptr;
    hperm_opts o;
    hperm_default_opts(&o);
    if (opts) {
        if (check_opts(opts)) return HPERM_E_INVALID;
        o = *opts;
    }
    hperm_ctx *c = new (std::nothrow) hperm_ctx();
    if (!c) return HPERM_E_NOMEM;
    c->opts = o;
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess) {
        delete c;
        return HPERM_E_DEVICE;
    }
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return HPERM_E_DEVICE;
        }
        c->own_stream = true;
    }
    c->dev.stream = c->stream;
    c->dev.opts = c->opts;
    c->dev.last_error.reserve(256);   // short error messages then need no allocation
    c->dev.tune = std::make_shared<TuneTable>();
    (void)noalloc_scratch(c->device);  // the no-allocation entry point's array, once per device
    *out = c;
    return HPERM_OK;
}

hperm_status hperm_ctx_create_host(const hperm_opts *opts, hperm_ctx **out) {
    if (!out) return HPERM_E_INVALID;
    *out = nullptr;
    hperm_opts o;
    hperm_default_opts(&o);
    if (opts) {
        if (check_opts(opts)) return HPERM_E_INVALID;
        o = *opts;
    }
    hperm_ctx *c = new (std::nothrow) hperm_ctx();
    if (!c) return HPERM_E_NOMEM;
    c->opts = o;
    c->host_only = true;
    *out = c;
    return HPERM_OK;
}


void hperm_ctx_destroy(hperm_ctx *c) {
    if (!c) return;
    if (c->host_only) {
        delete c;
        return;
    }
    hp::serve_shutdown(c);
    hp::dev_release(&c->dev);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

hperm_status hperm_ctx_get_opts(const hperm_ctx *c, hperm_opts *o) {
    if (!c || !o) return HPERM_E_INVALID;
    *o = c->opts;
    return HPERM_OK;
}

hperm_status hperm_ctx_set_opts(hperm_ctx *c, const hperm_opts *o) {
    if (!c || !o) return HPERM_E_INVALID;
    if (const char *why = check_opts(o)) return set_error(c, HPERM_E_INVALID, why);
    if (c->serving) return set_error(c, HPERM_E_INVALID, "the context is serving");
    c->opts = *o;
    return HPERM_OK;
}

hperm_status hperm_ctx_set_arena(hperm_ctx *c, void *dev_ptr, size_t bytes) {
    if (c && c->host_only) return set_error(c, HPERM_E_DEVICE, "host-only context");
    if (!c) return HPERM_E_INVALID;
    if (dev_ptr && bytes < 4096) return set_error(c, HPERM_E_INVALID, "arena too small");
    if (c->serving) return set_error(c, HPERM_E_INVALID, "the context is serving");
    (void)hipStreamSynchronize(c->stream);
    for (auto &b : c->dev.buf) {
        if (b.ptr && b.owned) (void)hipFree(b.ptr);
        b = DevBuf();
    }
    c->dev.arena = dev_ptr;
    c->dev.arena_bytes = dev_ptr ? bytes : 0;
    c->dev.resident_jobs = 0;
    c->dev.resident_list = 0;
    return HPERM_OK;
}

size_t hperm_ctx_arena_required(const hperm_ctx *c) { return c ? c->dev.arena_required : 0; }

static hperm_status expand_batch(hperm_ctx *c, int32_t count, const int32_t *n, const int64_t *rp_off,
                                 const int64_t *nz_off, const int32_t *row_ptr, const int32_t *col_idx,
                                 const uint32_t *val, hperm_jobs *j) {
    if (count < 0 || (count > 0 && (!n || !rp_off || !nz_off))) return set_error(c, HPERM_E_INVALID, "bad batch arrays");
    std::vector<CsrView> probs(count);
    for (int k = 0; k < count; ++k) {
        CsrView v{n[k], row_ptr ? row_ptr + rp_off[k] : nullptr, col_idx ? col_idx + nz_off[k] : nullptr,
                  val ? val + nz_off[k] : nullptr};
        const std::string why = validate_csr(v);
        if (!why.empty()) return set_error(c, HPERM_E_INVALID, "problem " + std::to_string(k) + ": " + why);
        probs[k] = v;
    }
    std::string err;
    const int rc = expand_problems(probs, expand_params(c->opts), &j->tab, &err);
    if (rc == -2) return set_error(c, HPERM_E_RANGE, err);
    if (rc == -3) return set_error(c, HPERM_E_NOMEM, err);
    if (rc) return set_error(c, HPERM_E_INVALID, err);
    j->id = next_jobs_id();
    return HPERM_OK;
}

// The host-expansion path of a batch (the caller holds call_mu).
static hperm_status batch_host_path(hperm_ctx *c, int32_t count, const int32_t *n, const int64_t *rp_off,
                                    const int64_t *nz_off, const int32_t *row_ptr, const int32_t *col_idx,
                                    const uint32_t *val, hperm_result *out) {
    const double t0 = now_s();
    // Problems are processed in up to four groups: the host expands group g + 1 on a thread of
    // its own while the device estimates and evaluates group g (each group has its own queue
    // in the chosen order). One group when the batch is small or runs one launch per job.
    const int groups = (c->opts.persistent && count >= 4) ? 4 : 1;
    std::vector<hperm_result> res(std::max(count, 1));   // copied to out only on success
    std::vector<hperm_jobs> tabs(groups);
    std::vector<hperm_status> est(groups, HPERM_OK);
    std::vector<double> t_exp(groups, 0.0);
    auto lo = [&](int g) { return (int)((int64_t)count * g / groups); };
    auto expand_group = [&](int g) {
        const double ta = now_s();
        est[g] = expand_batch(c, lo(g + 1) - lo(g), n + lo(g), rp_off + lo(g), nz_off + lo(g), row_ptr,
                              col_idx, val, &tabs[g]);
        t_exp[g] = now_s() - ta;
    };
    expand_group(0);
    double t_est = 0.0, t_rnw_all = 0.0;
    hperm_status s = est[0];
    for (int g = 0; g < groups && !s; ++g) {
        std::thread next;
        if (g + 1 < groups) next = std::thread(expand_group, g + 1);
        hperm_jobs &j = tabs[g];
        if (!j.tab.desc.empty() && (c->opts.order == HPERM_ORDER_ESTIMATE || c->opts.order == HPERM_ORDER_EXACT_COST)) {
            const double ta = now_s();
            s = estimate_jobs(&c->dev, &j, c->opts.trials, c->opts.seed);
            t_est += now_s() - ta;
        }
        double t_rnw = 0.0;
        if (!s) s = run_jobs(&c->dev, &j, c->opts.order, c->opts.persistent, nullptr, res.data() + lo(g), &t_rnw);
        t_rnw_all += t_rnw;
        j = hperm_jobs();   // release the group's host table
        if (next.joinable()) next.join();
        if (!s && g + 1 < groups) s = est[g + 1];
    }
    if (s) {
        if (c->dev.last_error.empty()) c->dev.last_error = "batch failed";
        return s;
    }
    const double t2 = now_s();
    double t_exp_all = 0.0;
    for (double t : t_exp) t_exp_all += t;
    for (int k = 0; k < count; ++k) {
        out[k] = res[k];
        out[k].t_expand_s = t_exp_all;
        out[k].t_estimate_s = t_est;
        out[k].t_rnw_s = t_rnw_all;
        out[k].t_total_s = t2 - t0;
    }
    return HPERM_OK;
}

hperm_status hperm_permanent_mod_batch_csr(hperm_ctx *c, int32_t count, const int32_t *n, const int64_t *rp_off,
                                           const int64_t *nz_off, const int32_t *row_ptr, const int32_t *col_idx,
                                           const uint32_t *val, uint32_t prime, uint64_t *residues) {
    if (c && c->host_only) return set_error(c, HPERM_E_DEVICE, "host-only context");
    if (!c || !residues) return HPERM_E_INVALID;
    if (c->serving) return set_error(c, HPERM_E_INVALID, "the context is serving");
    if (count < 0 || (count > 0 && (!n || !rp_off || !nz_off))) return set_error(c, HPERM_E_INVALID, "bad batch arrays");
    if (prime < 3 || prime >= (1u << 18) || !(prime & 1u)) return set_error(c, HPERM_E_INVALID, "an odd prime below 2^18");
    for (uint32_t d = 3; d * d <= prime; d += 2)
        if (prime % d == 0) return set_error(c, HPERM_E_INVALID, "the modulus must be prime");
    std::lock_guard<std::mutex> lk(c->call_mu);
    c->dev.last_error.clear();
    c->dev.opts = c->opts;
    c->dev.launches.clear();
    const int T = device_in_effect(c->opts) ? device_in_effect(c->opts) : 22;
    const int t = split_in_effect(c->opts) ? split_in_effect(c->opts) : 12;
    for (int k = 0; k < count; ++k) {
        CsrView v{n[k], row_ptr ? row_ptr + rp_off[k] : nullptr, col_idx ? col_idx + nz_off[k] : nullptr,
                  val ? val + nz_off[k] : nullptr};
        const std::string why = validate_csr(v);
        if (!why.empty()) return set_error(c, HPERM_E_INVALID, "problem " + std::to_string(k) + ": " + why);
        if (n[k] <= T || n[k] > HP_MAX_N || (uint64_t)n[k] * (prime - 1) >= (1u << 24))
            return set_error(c, HPERM_E_INVALID,
                             "modular evaluation: orders above the device expansion's, with n (p - 1) < 2^24");
    }
    const size_t budget = (size_t)(c->opts.device_expand_mib > 0 ? c->opts.device_expand_mib : 8192) << 20;
    std::vector<int> order_of((size_t)count);
    for (int k = 0; k < count; ++k) order_of[(size_t)k] = k;
    std::stable_sort(order_of.begin(), order_of.end(), [&](int x, int y) { return n[x] < n[y]; });
    for (size_t g0 = 0; g0 < order_of.size();) {   // problems of one order share one expansion
        size_t g1 = g0;
        while (g1 < order_of.size() && n[order_of[g1]] == n[order_of[g0]]) ++g1;
        std::vector<CsrView> grp;
        for (size_t q = g0; q < g1; ++q) {
            const int k = order_of[q];
            grp.push_back(CsrView{n[k], row_ptr + rp_off[k], col_idx + nz_off[k], val + nz_off[k]});
        }
        std::vector<U512> totals;
        DexpStats st;
        const std::vector<uint32_t> moduli(grp.size(), prime);
        hperm_status s = device_expand_group(&c->dev, grp, T, t, c->opts.s_leaf, budget, &totals, &st, nullptr, &moduli);
        if (s) return s;
        for (size_t q = g0; q < g1; ++q) residues[order_of[q]] = totals[q - g0].w[0];
        g0 = g1;
    }
    return HPERM_OK;
}

hperm_status hperm_permanent_batch_csr(hperm_ctx *c, int32_t count, const int32_t *n,
                                       const int64_t *rp_off, const int64_t *nz_off,
                                       const int32_t *row_ptr, const int32_t *col_idx,
                                       const uint32_t *val, hperm_result *out) {
    if (c && c->host_only) return set_error(c, HPERM_E_DEVICE, "host-only context");
    if (!c || !out) return HPERM_E_INVALID;
    if (c->serving) return set_error(c, HPERM_E_INVALID, "the context is serving");
    if (count < 0 || (count > 0 && (!n || !rp_off || !nz_off))) return set_error(c, HPERM_E_INVALID, "bad batch arrays");
    std::lock_guard<std::mutex> lk(c->call_mu);
    c->dev.last_error.clear();
    c->dev.opts = c->opts;
    // problems for the device expansion, one at a time; the others in one host-path batch
    std::vector<int> dev_idx, host_idx;
    for (int k = 0; k < count; ++k) {
        CsrView v{n[k], row_ptr ? row_ptr + rp_off[k] : nullptr, col_idx ? col_idx + nz_off[k] : nullptr,
                  val ? val + nz_off[k] : nullptr};
        const std::string why = validate_csr(v);
        if (!why.empty()) return set_error(c, HPERM_E_INVALID, "problem " + std::to_string(k) + ": " + why);
        (device_path(c->opts, v) ? dev_idx : host_idx).push_back(k);
    }
    std::vector<hperm_result> res(count);
    std::vector<int> res_idx;   // problems for the residue evaluation
    if (!host_idx.empty()) {
        std::vector<int32_t> hn;
        std::vector<int64_t> hr, hz;
        for (int k : host_idx) {
            hn.push_back(n[k]);
            hr.push_back(rp_off[k]);
            hz.push_back(nz_off[k]);
        }
        std::vector<hperm_result> hres(host_idx.size());
        hperm_status s = batch_host_path(c, (int32_t)host_idx.size(), hn.data(), hr.data(), hz.data(), row_ptr, col_idx,
                                         val, hres.data());
        if (s == HPERM_E_RANGE) {
            // one problem at a time: those out of the host path's range (the 2^180 bound, or an
            // expanded entry past 2^22) go to the residue evaluation where it takes them
            for (size_t q = 0; q < host_idx.size(); ++q) {
                const int k = host_idx[q];
                s = batch_host_path(c, 1, hn.data() + q, hr.data() + q, hz.data() + q, row_ptr, col_idx, val,
                                    hres.data() + q);
                if (s == HPERM_E_RANGE && residue_path(c->opts, n[k])) {
                    res_idx.push_back(k);
                    s = HPERM_OK;
                    continue;
                }
                if (s) return s;
                res[k] = hres[q];
            }
            c->dev.last_error.clear();
        } else if (s) {
            return s;
        } else {
            for (size_t q = 0; q < host_idx.size(); ++q) res[host_idx[q]] = hres[q];
        }
        if (dev_idx.empty() && res_idx.empty()) {
            for (int k = 0; k < count; ++k) out[k] = res[k];
            return HPERM_OK;
        }
    }
    if (host_idx.empty()) c->dev.launches.clear();
    const size_t budget = (size_t)(c->opts.device_expand_mib > 0 ? c->opts.device_expand_mib : 8192) << 20;
    // problems of one order share one device expansion
    std::vector<int> order_of(dev_idx);
    std::stable_sort(order_of.begin(), order_of.end(), [&](int x, int y) { return n[x] < n[y]; });
    for (size_t g0 = 0; g0 < order_of.size();) {
        size_t g1 = g0;
        while (g1 < order_of.size() && n[order_of[g1]] == n[order_of[g0]]) ++g1;
        const double t0 = now_s();
        std::vector<CsrView> grp;
        for (size_t q = g0; q < g1; ++q) {
            const int k = order_of[q];
            grp.push_back(CsrView{n[k], row_ptr + rp_off[k], col_idx + nz_off[k], val + nz_off[k]});
        }
        std::vector<U512> totals;
        DexpStats st;
        hperm_status s = device_expand_group(&c->dev, grp, device_in_effect(c->opts), split_in_effect(c->opts),
                                             c->opts.s_leaf, budget, &totals, &st);
        if (s == HPERM_E_RANGE) {   // an expanded entry past 2^22: the residue evaluation
            for (size_t q = g0; q < g1; ++q) res_idx.push_back(order_of[q]);
            c->dev.last_error.clear();
            g0 = g1;
            continue;
        }
        if (s) return s;
        const double t1 = now_s();
        for (size_t q = g0; q < g1; ++q) {
            hperm_result &r = res[order_of[q]];
            memset(&r, 0, sizeof(r));
            fill_result(totals[q - g0], &r);
            r.n_jobs = (int32_t)std::min<uint64_t>(st.jobs, 0x7fffffff);   // the group's figures
            r.max_m = device_in_effect(c->opts);
            r.arith_mask = 1 << (HPERM_ARITH_W64);
            r.subset_terms = st.leaf_terms;
            r.t_rnw_s = st.split_s;
            r.t_expand_s = st.total_s - st.split_s;
            r.t_total_s = t1 - t0;
        }
        hperm_launch_stat ls{};
        ls.ring = HP_W64;
        ls.bucket = bucket_of(device_in_effect(c->opts));
        ls.n_jobs = (int32_t)std::min<uint64_t>(st.jobs, 0x7fffffff);
        ls.persistent = 1;
        ls.variant = 4;
        ls.reserved = (int32_t)(g1 - g0);
        ls.items = st.nodes;
        ls.terms = st.leaf_terms;
        ls.row_updates = st.launches;
        ls.ms = st.total_s * 1e3;
        ls.leaves = st.leaves;
        ls.leaf_terms = st.leaf_terms;
        ls.splits = st.splits;
        ls.split_stops = st.split_stops;
        ls.deferred = st.deferred;
        ls.deferred_bound = st.deferred_bound;
        ls.alg_slots = st.split_s * 1e3;   // the device H_per launches' share of ms
        c->dev.launches.push_back(ls);
        g0 = g1;
    }
    // the residue evaluation, problems of one order together
    std::stable_sort(res_idx.begin(), res_idx.end(), [&](int x, int y) { return n[x] < n[y]; });
    for (size_t g0 = 0; g0 < res_idx.size();) {
        size_t g1 = g0;
        while (g1 < res_idx.size() && n[res_idx[g1]] == n[res_idx[g0]]) ++g1;
        const double t0 = now_s();
        std::vector<CsrView> grp;
        for (size_t q = g0; q < g1; ++q) {
            const int k = res_idx[q];
            grp.push_back(CsrView{n[k], row_ptr + rp_off[k], col_idx + nz_off[k], val + nz_off[k]});
        }
        std::vector<U512> totals;
        DexpStats st;
        int np = 0;
        const hperm_status s = device_expand_residues(&c->dev, grp, device_in_effect(c->opts), split_in_effect(c->opts),
                                                      c->opts.s_leaf, budget, &totals, &st, &np);
        if (s) return s;
        const double t1 = now_s();
        for (size_t q = g0; q < g1; ++q) {
            hperm_result &r = res[res_idx[q]];
            memset(&r, 0, sizeof(r));
            fill_result(totals[q - g0], &r);
            r.n_jobs = (int32_t)std::min<uint64_t>(st.jobs, 0x7fffffff);   // the group's figures, all primes
            r.max_m = device_in_effect(c->opts);
            r.arith_mask = 1 << (HPERM_ARITH_RES);
            r.subset_terms = st.leaf_terms;
            r.t_rnw_s = st.split_s;
            r.t_expand_s = st.total_s - st.split_s;
            r.t_total_s = t1 - t0;
        }
        hperm_launch_stat ls{};
        ls.ring = HP_RES;
        ls.bucket = bucket_of(device_in_effect(c->opts));
        ls.n_jobs = (int32_t)std::min<uint64_t>(st.jobs, 0x7fffffff);
        ls.persistent = 1;
        ls.variant = 5;
        ls.reserved = (int32_t)(g1 - g0);
        ls.items = st.nodes;
        ls.terms = st.leaf_terms;
        ls.row_updates = np;
        ls.ms = st.total_s * 1e3;
        ls.leaves = st.leaves;
        ls.leaf_terms = st.leaf_terms;
        ls.splits = st.splits;
        ls.split_stops = st.split_stops;
        ls.deferred = st.deferred;
        ls.deferred_bound = st.deferred_bound;
        ls.alg_slots = st.split_s * 1e3;
        c->dev.launches.push_back(ls);
        g0 = g1;
    }
    for (int k = 0; k < count; ++k) out[k] = res[k];
    return HPERM_OK;
}

hperm_status hperm_device_expand_sample(hperm_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                        const uint32_t *val, int32_t max_jobs, int32_t stop_early, uint32_t *mats,
                                        hperm_result *values, int32_t *n_sampled, hperm_result *total) {
    if (c && c->host_only) return set_error(c, HPERM_E_DEVICE, "host-only context");
    if (!c || !n_sampled || !total || max_jobs < 0 || (max_jobs > 0 && (!mats || !values))) return HPERM_E_INVALID;
    if (c->serving) return set_error(c, HPERM_E_INVALID, "the context is serving");
    const int T = device_in_effect(c->opts), t = split_in_effect(c->opts);
    if (T <= 0 || t <= 0)
        return set_error(c, HPERM_E_INVALID, "device_expand must exceed a split_order in effect");
    CsrView v{n, row_ptr, col_idx, val};
    const std::string why = validate_csr(v);
    if (!why.empty()) return set_error(c, HPERM_E_INVALID, why);
    if (n <= T) return set_error(c, HPERM_E_INVALID, "the order must exceed device_expand");
    std::lock_guard<std::mutex> lk(c->call_mu);
    c->dev.last_error.clear();
    c->dev.opts = c->opts;
    const size_t budget = (size_t)(c->opts.device_expand_mib > 0 ? c->opts.device_expand_mib : 8192) << 20;
    DexpSample smp;
    smp.max_jobs = (uint64_t)max_jobs;
    smp.stop_early = stop_early != 0;
    U512 tot;
    DexpStats st;
    const double t0 = now_s();
    hperm_status s = device_expand_problem(&c->dev, v, T, t, c->opts.s_leaf, budget, &tot, &st, &smp);
    if (s) return s;
    const size_t k = smp.vals.size();
    std::copy(smp.mats.begin(), smp.mats.end(), mats);
    for (size_t q = 0; q < k; ++q) {
        memset(&values[q], 0, sizeof(hperm_result));
        fill_result(smp.vals[q], &values[q]);
        values[q].n_jobs = 1;
        values[q].max_m = T;
    }
    *n_sampled = (int32_t)k;
    memset(total, 0, sizeof(*total));
    if (smp.complete) fill_result(tot, total);
    total->n_jobs = (int32_t)std::min<uint64_t>(st.jobs, 0x7fffffff);
    total->max_m = smp.complete ? T : 0;   // 0: stopped early, the value is not per(A)
    total->subset_terms = st.leaf_terms;
    total->t_rnw_s = st.split_s;
    total->t_total_s = now_s() - t0;
    return HPERM_OK;
}

hperm_status hperm_tree_estimate(const hperm_opts *opts, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                 const uint32_t *val, int32_t samples, uint64_t seed, double *nodes, double *leaves) {
    if (!nodes || !leaves || samples < 1) return HPERM_E_INVALID;
    hperm_opts o;
    hperm_default_opts(&o);
    if (opts) {
        if (check_opts(opts)) return HPERM_E_INVALID;
        o = *opts;
    }
    CsrView v{n, row_ptr, col_idx, val};
    if (!validate_csr(v).empty()) return HPERM_E_INVALID;
    const int t = split_in_effect(o) > 0 ? split_in_effect(o) : o.m_cut;
    const int T = device_in_effect(o) > 0 ? device_in_effect(o) : o.m_cut;
    return estimate_tree(v, std::max(T, t), t, o.s_leaf, samples, seed, nodes, leaves) ? HPERM_E_RANGE : HPERM_OK;
}

hperm_status hperm_permanent_csr(hperm_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                 const uint32_t *val, hperm_result *out) {
    const int64_t z = 0;
    return hperm_permanent_batch_csr(c, 1, &n, &z, &z, row_ptr, col_idx, val, out);
}

hperm_status hperm_permanent_dense(hperm_ctx *c, int32_t n, const uint32_t *a, hperm_result *out) {
    if (!c || !out) return HPERM_E_INVALID;
    if (n < 0 || n > HP_MAX_N) return set_error(c, HPERM_E_INVALID, "n must be in [0, 128]");
    if (n > 0 && !a) return set_error(c, HPERM_E_INVALID, "a is null");
    std::vector<int32_t> rp(n + 1, 0), ci;
    std::vector<uint32_t> v;
    for (int i = 0; i < n; ++i) {
        for (int jj = 0; jj < n; ++jj)
            if (a[(int64_t)i * n + jj]) {
                ci.push_back(jj);
                v.push_back(a[(int64_t)i * n + jj]);
            }
        rp[i + 1] = (int32_t)ci.size();
    }
    return hperm_permanent_csr(c, n, rp.data(), ci.data(), v.data(), out);
}

hperm_status hperm_expand_batch_csr(hperm_ctx *c, int32_t count, const int32_t *n, const int64_t *rp_off,
                                    const int64_t *nz_off, const int32_t *row_ptr, const int32_t *col_idx,
                                    const uint32_t *val, hperm_jobs **out) {
    if (!c || !out) return HPERM_E_INVALID;
    *out = nullptr;
    hperm_jobs *j = new (std::nothrow) hperm_jobs();
    if (!j) return HPERM_E_NOMEM;
    hperm_status s = expand_batch(c, count, n, rp_off, nz_off, row_ptr, col_idx, val, j);
    if (s) {
        delete j;
        return s;
    }
    *out = j;
    return HPERM_OK;
}

hperm_status hperm_jobs_from_dense(hperm_ctx *c, int32_t count, const int32_t *m, const int64_t *off,
                                   const uint32_t *a, hperm_jobs **out) {
    if (!c || !out || count < 0 || (count > 0 && (!m || !off || !a))) return HPERM_E_INVALID;
    *out = nullptr;
    hperm_jobs *j = new (std::nothrow) hperm_jobs();
    if (!j) return HPERM_E_NOMEM;
    std::string err;
    const int rc = jobs_from_dense(count, m, off, a, expand_params(c->opts), &j->tab, &err);
    if (rc) {
        delete j;
        return set_error(c, rc == -2 ? HPERM_E_RANGE : rc == -3 ? HPERM_E_NOMEM : HPERM_E_INVALID, err);
    }
    j->id = next_jobs_id();
    *out = j;
    return HPERM_OK;
}

hperm_status hperm_jobs_info(const hperm_jobs *j, int32_t *n_jobs, int32_t *n_problems) {
    if (!j || !n_jobs || !n_problems) return HPERM_E_INVALID;
    *n_jobs = (int32_t)j->tab.desc.size();
    *n_problems = j->tab.n_problems;
    return HPERM_OK;
}

hperm_status hperm_jobs_describe(const hperm_jobs *j, int32_t *m, int32_t *problem, int32_t *arith,
                                 uint64_t *terms) {
    if (!j) return HPERM_E_INVALID;
    for (size_t k = 0; k < j->tab.desc.size(); ++k) {
        const JobDesc &d = j->tab.desc[k];
        if (m) m[k] = d.m;
        if (problem) problem[k] = (int32_t)d.problem;
        if (arith) arith[k] = d.arith + 1;
        if (terms) terms[k] = 1ull << (d.m - 1);
    }
    return HPERM_OK;
}

hperm_status hperm_jobs_matrix(const hperm_jobs *j, int32_t job, uint32_t *a) {
    if (!j || !a || job < 0 || (size_t)job >= j->tab.desc.size()) return HPERM_E_INVALID;
    const JobDesc &d = j->tab.desc[(size_t)job];
    const int m = d.m;
    const uint32_t *blk = j->tab.data.data() + hp_data_index(d);
    std::fill(a, a + (size_t)m * m, 0u);
    for (int g = 0; g + 1 < m; ++g)   // Gray column g: entries (2 b_ig << 8) | i
        for (uint32_t e = blk[m + g]; e < blk[m + g + 1]; ++e) {
            const uint32_t w = blk[3 * m + e];
            a[(size_t)(w & 0xffu) * m + g] = w >> 9;
        }
    for (int i = 0; i < m; ++i) {     // fixed column: b_i = base_i + sum of the Gray entries
        int64_t v = (int32_t)blk[i];
        for (int g = 0; g + 1 < m; ++g) v += a[(size_t)i * m + g];
        a[(size_t)i * m + m - 1] = (uint32_t)v;
    }
    return HPERM_OK;
}

hperm_status hperm_estimate(hperm_ctx *c, hperm_jobs *j, int32_t trials, uint64_t seed, float *keys) {
    if (c && c->host_only) return set_error(c, HPERM_E_DEVICE, "host-only context");
    if (!c || !j) return HPERM_E_INVALID;
    if (c->serving) return set_error(c, HPERM_E_INVALID, "the context is serving");
    std::lock_guard<std::mutex> lk(c->call_mu);
    c->dev.opts = c->opts;
    hperm_status s = estimate_jobs(&c->dev, j, trials, seed);
    if (s) return s;
    if (keys) std::copy(j->keys.begin(), j->keys.end(), keys);
    return HPERM_OK;
}

hperm_status hperm_run_jobs(hperm_ctx *c, hperm_jobs *j, int32_t order, int32_t persistent,
                            hperm_result *per_job, hperm_result *totals) {
    if (c && c->host_only) return set_error(c, HPERM_E_DEVICE, "host-only context");
    if (!c || !j || !totals) return HPERM_E_INVALID;
    if (c->serving) return set_error(c, HPERM_E_INVALID, "the context is serving");
    std::lock_guard<std::mutex> lk(c->call_mu);
    const double t0 = now_s();
    double t_rnw = 0.0;
    c->dev.opts = c->opts;
    hperm_status s = run_jobs(&c->dev, j, order, persistent, per_job, totals, &t_rnw);
    if (s) return s;
    const double t1 = now_s();
    for (int p = 0; p < j->tab.n_problems; ++p) totals[p].t_total_s = t1 - t0;
    return HPERM_OK;
}

void hperm_jobs_free(hperm_jobs *j) { delete j; }

hperm_status hperm_jobs_cycles(const hperm_jobs *j, uint64_t *cycles) {
    if (!j || !cycles || !j->has_cycles || j->cycles.size() != j->tab.desc.size()) return HPERM_E_INVALID;
    std::copy(j->cycles.begin(), j->cycles.end(), cycles);
    return HPERM_OK;
}

hperm_status hperm_last_launches(const hperm_ctx *c, hperm_launch_stat *out, int32_t max, int32_t *n) {
    if (!c || !n || max < 0 || (max > 0 && !out)) return HPERM_E_INVALID;
    const int32_t k = (int32_t)std::min<size_t>((size_t)max, c->dev.launches.size());
    for (int32_t i = 0; i < k; ++i) out[i] = c->dev.launches[i];
    *n = (int32_t)c->dev.launches.size();
    return HPERM_OK;
}

const char *hperm_status_string(hperm_status s) {
    switch (s) {
        case HPERM_OK: return "ok";
        case HPERM_NOT_READY: return "not ready";
        case HPERM_E_INVALID: return "invalid argument";
        case HPERM_E_RANGE: return "out of the supported integer range";
        case HPERM_E_DEVICE: return "device error";
        case HPERM_E_NOMEM: return "out of memory";
        case HPERM_E_BUSY: return "busy";
        case HPERM_E_CANCELLED: return "cancelled";
        case HPERM_E_TIMEOUT: return "timed out";
        case HPERM_E_INTERNAL: return "internal integrity check failed";
        case HPERM_E_TOOBIG: return "estimated work beyond the serving limit";
    }
    return "unknown status";
}

const char *hperm_last_error(const hperm_ctx *c) { return c ? c->dev.last_error.c_str() : ""; }

}  // extern "C"
