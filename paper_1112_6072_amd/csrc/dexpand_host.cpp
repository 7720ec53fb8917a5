// Host driver of the device expansion (dexpand.hip) and of the device continuation of H_per on
// its nodes (split.hip): per(A) of one problem with every node of the expansion tree built on
// the GPU.
//
// Level o of the tree (nodes of order o) has a buffer of W words and N node offsets. The root
// (order n) is uploaded; a level is expanded chunk by chunk into the level below, and each
// chunk's children are processed completely (recursively, down to the job order T) before the
// next chunk of the level is expanded into the same buffer, so the memory in use is bounded by
// the level buffers whatever the size of the tree. At order T the nodes are the jobs of the
// device continuation of H_per, which splits them down to order t and evaluates the leaves;
// every such launch sums into a staging accumulator that is checked (integrity counters,
// record overflow) before its value joins the problem's exact total on the host.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"
#include "expand.h"
#include "kernels.h"

namespace hp {

hipError_t launch_dexp_plan(const uint32_t *lvl, const uint64_t *off, uint64_t first, uint32_t n, uint32_t *keys,
                            uint64_t *packed, hipStream_t s);
size_t dexp_scan_tiles(uint32_t n);
hipError_t launch_dexp_scan(const uint64_t *in, uint32_t n, uint64_t *tile_sums, uint64_t *out, uint64_t *grand,
                            hipStream_t s);
// flags[0] |= 1 on a range error.
hipError_t launch_dexp_write(const uint32_t *lvl, const uint64_t *off, uint64_t first, uint32_t n, const uint32_t *keys,
                             const uint64_t *place, uint32_t *out, uint64_t *out_off, unsigned long long *flags,
                             const uint32_t *primes, hipStream_t s);

namespace {

// Small device block read back after each step: scan total, range flag, split counters and the
// staging accumulator of the last launch.
struct Misc {
    unsigned long long grand;          // packed (children << 36 | words) of the last scan
    unsigned long long flags;          // bit 0: an entry or row sum out of range
    unsigned long long pad;
    unsigned long long head;           // queue counter of the split launch
    unsigned long long stats[HP_SPLIT_STATS];
};

struct Plan {
    int n = 0, T = 0, t = 0, s_leaf = 5;
    const uint32_t *modps = nullptr;   // modular mode: each problem's prime, on the device (nullptr: exact)
    uint64_t W = 0, N = 0;             // words and node offsets per level
    uint32_t *levels = nullptr;        // level o at levels + (o - T) * W
    uint64_t *offs = nullptr;          // level o's offsets at offs + (o - T) * N
    uint32_t *keys = nullptr;          // plan of a chunk (N / 2 entries)
    uint64_t *packed = nullptr, *place = nullptr, *tiles = nullptr;
    Misc *misc = nullptr;              // device
    ProbAcc *probs = nullptr;          // device: one split launch's sums, one per problem
    int nprob = 1;
    void *wide = nullptr;
    uint64_t wide_entries = 0;
    std::vector<uint32_t> maxw;        // per level: words per node to size its chunks by
};

}  // namespace

struct DexpRun {
    Dev *c;
    Plan P;
    std::vector<U512> total;           // per problem of the group
    DexpStats st;
    std::string err;
    hperm_status status = HPERM_OK;
    // the first sample_max jobs (tree order): dense T x T matrices and their values
    uint64_t sample_max = 0;
    bool stop_after_sample = false;
    std::vector<uint32_t> *sample_mats = nullptr;
    std::vector<U512> *sample_vals = nullptr;
    bool stopped = false;

    hperm_status fail(hperm_status s, const std::string &m) {
        status = s;
        err = m;
        return s;
    }
    hperm_status hip(hipError_t e, const char *what) {
        if (e == hipSuccess) return HPERM_OK;
        return fail(e == hipErrorOutOfMemory ? HPERM_E_NOMEM : HPERM_E_DEVICE,
                    std::string(what) + ": " + hipGetErrorString(e));
    }

    uint32_t *level(int o) const { return P.levels + (size_t)(o - P.T) * P.W; }
    uint64_t *offs(int o) const { return P.offs + (size_t)(o - P.T) * P.N; }

    // The jobs of level T [0, n): the device continuation of H_per, checked and summed.
    hperm_status run_jobs(uint64_t n) {
        hipStream_t s = c->stream;
        Misc *m = P.misc;
        Misc h;
        const uint64_t have = sample_vals ? sample_vals->size() : 0;
        const uint64_t take = sample_max > have ? std::min<uint64_t>(sample_max - have, n) : 0;
        JobAcc *accs = nullptr;
        if (take) {   // per-node values of this launch are kept (the first jobs of the tree)
            hperm_status r = ensure_buf(c, B_ACCS, n * sizeof(JobAcc));
            if (r) return fail(r, c->last_error);
            if (c->arena) return fail(HPERM_E_INVALID, "sampling device jobs needs library-owned memory");
            accs = (JobAcc *)c->buf[B_ACCS].ptr;
            r = hip(launch_fill_u64((unsigned long long *)accs, n * (sizeof(JobAcc) / 8), 0ull, s), "clear accumulators");
            if (r) return r;
        }
        std::vector<ProbAcc> hp_((size_t)P.nprob);
        for (int attempt = 0;; ++attempt) {
            hperm_status r = hip(launch_fill_u64((unsigned long long *)&m->head,
                                                 (sizeof(Misc) - offsetof(Misc, head)) / 8, 0ull, s),
                                 "clear split counters");
            if (r) return r;
            r = hip(launch_fill_u64((unsigned long long *)P.probs, (uint64_t)P.nprob * (sizeof(ProbAcc) / 8), 0ull, s),
                    "clear problem sums");
            if (r) return r;
            const double t0 = now_s();
            if (accs && attempt) {
                r = hip(launch_fill_u64((unsigned long long *)accs, n * (sizeof(JobAcc) / 8), 0ull, s),
                        "clear accumulators");
                if (r) return r;
            }
            r = hip(launch_split_nodes(level(P.T), offs(P.T), (uint32_t)n, P.t, P.T, P.s_leaf, &m->head, accs,
                                       P.probs, m->stats, P.wide, P.wide_entries, P.modps, s),
                    "device H_per launch");
            if (r) return r;
            r = hip(hipMemcpyAsync(&h, m, sizeof(Misc), hipMemcpyDeviceToHost, s), "download split results");
            if (r) return r;
            r = hip(hipMemcpyAsync(hp_.data(), P.probs, hp_.size() * sizeof(ProbAcc), hipMemcpyDeviceToHost, s),
                    "download problem sums");
            if (r) return r;
            r = hip(hipStreamSynchronize(s), "device H_per");
            if (r) return r;
            st.split_s += now_s() - t0;
            // the expansion's range flag (set by any write kernel of the levels above): checked
            // here, at the first synchronisation after those writes, before any value is used
            if (h.flags & 1) return fail(HPERM_E_RANGE, "an expanded entry reached 2^22 or a row sum 2^24");
            if (h.stats[6]) return fail(HPERM_E_INTERNAL, "device H_per: a leaf value failed its integrity check");
            if (!h.stats[5]) break;
            // the record buffer overflowed: the launch's sum is dropped and the launch repeated
            // with room for every deferred leaf it reported
            if (attempt >= 2) return fail(HPERM_E_INTERNAL, "device H_per: leaf records lost");
            const uint64_t need = h.stats[4] + 1024;
            r = ensure_buf(c, B_SPLIT_WIDE, split_wide_bytes(need));
            if (r) return fail(r, c->last_error);
            if (!c->arena) {   // a fresh allocation moves only this buffer
                P.wide = c->buf[B_SPLIT_WIDE].ptr;
                P.wide_entries = need;
            } else {
                return fail(HPERM_E_NOMEM, "device H_per: the arena cannot hold the leaf records");
            }
            ++st.relaunches;
        }
        if (take) {
            std::vector<uint64_t> off(take);
            std::vector<JobAcc> acc(take);
            hperm_status r = hip(hipMemcpy(off.data(), offs(P.T), take * 8, hipMemcpyDeviceToHost), "download offsets");
            if (r) return r;
            r = hip(hipMemcpy(acc.data(), accs, take * sizeof(JobAcc), hipMemcpyDeviceToHost), "download values");
            if (r) return r;
            const int T = P.T;
            std::vector<uint32_t> node(hp_node_words(T, T * T));
            for (uint64_t q = 0; q < take; ++q) {
                r = hip(hipMemcpy(node.data(), level(T) + off[q], 16, hipMemcpyDeviceToHost), "download node header");
                if (r) return r;
                const uint32_t words = hp_node_words((int)(node[0] & 0xffu), (int)(node[0] >> 8));
                if ((node[0] & 0xffu) != (uint32_t)T || words > node.size())
                    return fail(HPERM_E_INTERNAL, "device expansion: a job node has the wrong order");
                r = hip(hipMemcpy(node.data(), level(T) + off[q], words * 4, hipMemcpyDeviceToHost), "download node");
                if (r) return r;
                const size_t base = sample_mats->size();
                sample_mats->resize(base + (size_t)T * T, 0u);
                const uint32_t *ent = node.data() + 4 + (T + 3) / 4;
                uint32_t e = 0;
                for (int i = 0; i < T; ++i) {
                    const uint32_t len = (node[4 + i / 4] >> (8 * (i & 3))) & 0xffu;
                    for (uint32_t z = 0; z < len; ++z, ++e) (*sample_mats)[base + (size_t)i * T + (ent[e] & 0xffu)] = ent[e] >> 8;
                }
                U512 v;
                for (int l = 3; l >= 0; --l) {
                    U512 t;
                    t.w[0] = acc[q].l[l];
                    for (int z = 0; z < l; ++z) t.mul_u64(1ull << 32);
                    v.add(t);
                }
                sample_vals->push_back(v);
            }
            if (stop_after_sample && sample_vals->size() >= sample_max) stopped = true;
        }
        for (int k = 0; k < P.nprob; ++k) total[(size_t)k].add(prob_value(hp_[(size_t)k]));
        st.jobs += n;
        st.launches++;
        st.leaves += h.stats[0];
        st.leaf_terms += h.stats[1];
        st.splits += h.stats[2];
        st.split_stops += h.stats[3];
        st.deferred += h.stats[4];
        st.deferred_bound += h.stats[7];
        return HPERM_OK;
    }

    // Expand nodes [lo, hi) of level o (o > T) into level o - 1 chunk by chunk, each chunk's
    // subtree finished before the next.
    hperm_status process(int o, uint64_t lo, uint64_t hi) {
        hipStream_t s = c->stream;
        uint64_t k = lo;
        while (k < hi) {
            const uint64_t mw = std::max<uint64_t>(P.maxw[o - P.T], 8);
            uint64_t chunk = std::min<uint64_t>(hi - k, std::min<uint64_t>(P.N / 2, P.W / (2 * mw)));
            chunk = std::max<uint64_t>(chunk, 1);
            for (;;) {
                unsigned long long tot[2];
                hperm_status r = hip(launch_dexp_plan(level(o), offs(o), k, (uint32_t)chunk, P.keys, P.packed, s),
                                     "expansion plan");
                if (r) return r;
                r = hip(launch_dexp_scan(P.packed, (uint32_t)chunk, P.tiles, P.place, (uint64_t *)&P.misc->grand, s),
                        "expansion scan");
                if (r) return r;
                r = hip(hipMemcpyAsync(tot, &P.misc->grand, sizeof(tot), hipMemcpyDeviceToHost, s),
                        "download expansion totals");
                if (r) return r;
                r = hip(hipStreamSynchronize(s), "expansion plan");
                if (r) return r;
                const uint64_t kids = tot[0] >> 36, words = tot[0] & ((1ull << 36) - 1);
                if (kids <= P.N && words <= P.W) {
                    st.nodes += kids;
                    st.max_level_nodes = std::max<uint64_t>(st.max_level_nodes, kids);
                    if (kids) {
                        // the write's range flag is read at the next synchronisation (the
                        // continuation's results, or the end of the expansion): an entry out of
                        // range changes values only, never the tree's shape or its addresses
                        r = hip(launch_dexp_write(level(o), offs(o), k, (uint32_t)chunk, P.keys, P.place,
                                                  level(o - 1), offs(o - 1), &P.misc->flags, P.modps, s),
                                "expansion write");
                        if (r) return r;
                        // chunks of the next level are sized by the average room its nodes were
                        // given (the parent's words); a plan that outgrows a buffer halves them
                        P.maxw[o - 1 - P.T] = (uint32_t)((words + kids - 1) / kids);
                        r = o - 1 == P.T ? run_jobs(kids) : process(o - 1, 0, kids);
                        if (r) return r;
                        if (stopped) return HPERM_OK;
                    }
                    break;
                }
                if (chunk == 1) return fail(HPERM_E_NOMEM, "device expansion: one node's children exceed a level buffer");
                chunk /= 2;   // nodes with more than two children (lines of five or more nonzeros)
            }
            k += chunk;
        }
        return HPERM_OK;
    }
};

hperm_status device_expand_group(Dev *c, const std::vector<CsrView> &probs_in, int T, int t, int s_leaf,
                                 size_t budget_bytes, std::vector<U512> *out, DexpStats *stats, DexpSample *sample,
                                 const std::vector<uint32_t> *moduli) {
    // modular mode: each input's entries reduced modulo its prime (zeros dropped) before packing
    std::vector<std::vector<int32_t>> mrp, mci;
    std::vector<std::vector<uint32_t>> mva;
    std::vector<CsrView> reduced;
    if (moduli) {
        if (moduli->size() != probs_in.size()) return set_error(c, HPERM_E_INVALID, "modular device expansion: one prime per problem");
        for (size_t k = 0; k < probs_in.size(); ++k) {   // entries below p keep every row sum below 2^24
            const uint32_t modp = (*moduli)[k];
            if (modp < 3 || modp >= (1u << 18) || (uint64_t)probs_in[k].n * (modp - 1) >= (1u << 24))
                return set_error(c, HPERM_E_INVALID, "modular device expansion: a prime p below 2^18 with n (p - 1) < 2^24");
        }
        for (size_t k = 0; k < probs_in.size(); ++k) {
            const CsrView &a = probs_in[k];
            const uint32_t modp = (*moduli)[k];
            mrp.emplace_back();
            mci.emplace_back();
            mva.emplace_back();
            mrp.back().push_back(0);
            for (int i = 0; i < a.n; ++i) {
                for (int32_t e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e)
                    if (a.val[e] % modp) {
                        mci.back().push_back(a.col_idx[e]);
                        mva.back().push_back(a.val[e] % modp);
                    }
                mrp.back().push_back((int32_t)mci.back().size());
            }
            mci.back().push_back(0);   // non-empty arrays
            mva.back().push_back(0);
        }
        for (size_t k = 0; k < probs_in.size(); ++k)
            reduced.push_back(CsrView{probs_in[k].n, mrp[k].data(), mci[k].data(), mva[k].data()});
    }
    const std::vector<CsrView> &probs = moduli ? reduced : probs_in;
    DexpRun run{c, Plan{}, {}, DexpStats{}, std::string(), HPERM_OK};
    if (sample) {
        run.sample_max = sample->max_jobs;
        run.stop_after_sample = sample->stop_early;
        run.sample_mats = &sample->mats;
        run.sample_vals = &sample->vals;
        sample->mats.clear();
        sample->vals.clear();
    }
    Plan &P = run.P;
    const int count = (int)probs.size();
    out->assign((size_t)count, U512());
    if (count == 0) return HPERM_OK;
    const int n = probs[0].n;
    if (n <= T || T > HP_SPLIT_MAX_M || t < HP_SPLIT_MIN_T || t >= T)
        return set_error(c, HPERM_E_INVALID, "device expansion: needs t < T <= 24 < n");
    // the roots (problem k's carries k), their bounds (rows, columns and Bregman's for 0-1
    // inputs); problems with a zero line are 0 without device work
    std::vector<uint32_t> roots;
    std::vector<uint64_t> root_off;
    std::vector<double> bounds((size_t)count, 0.0);
    std::vector<int> live;
    uint32_t maxroot = 0;
    for (int k = 0; k < count; ++k) {
        if (probs[(size_t)k].n != n) return set_error(c, HPERM_E_INVALID, "device expansion: a group has one order");
        std::vector<uint32_t> root;
        const int rc = pack_root_node(probs[(size_t)k], &root, &bounds[(size_t)k]);
        if (rc == 1) continue;
        if (rc) return set_error(c, rc == -2 ? HPERM_E_RANGE : HPERM_E_INVALID, "device expansion: input out of range");
        if (!moduli && bounds[(size_t)k] > 102.0)
            return set_error(c, HPERM_E_RANGE, "device expansion: the permanent bound exceeds 2^102");
        root[2] = (uint32_t)k;
        root_off.push_back(roots.size());
        roots.insert(roots.end(), root.begin(), root.end());
        maxroot = std::max<uint32_t>(maxroot, (uint32_t)root.size());
        live.push_back(k);
    }
    if (live.empty()) {
        if (stats) *stats = run.st;
        if (sample) sample->complete = true;
        return HPERM_OK;
    }
    run.total.assign((size_t)count, U512());
    P.n = n;
    P.T = T;
    P.t = t;
    P.s_leaf = s_leaf;
    P.nprob = count;
    const int L = n - T + 1;
    // per level: 7/8 of its share in words, 1/8 in 8-byte offsets; the plan arrays for half a
    // level's offsets; the record buffer
    const size_t share = budget_bytes / (size_t)(L + 1);
    P.W = std::min<uint64_t>((share * 7 / 8) / 4, (uint64_t)1 << 29);
    P.N = std::max<uint64_t>(std::min<uint64_t>((share / 8) / 8, (uint64_t)1 << 26), 64);
    P.W = std::max<uint64_t>(P.W, 2 * (uint64_t)roots.size() + 64);
    P.N = std::max<uint64_t>(P.N, 2 * (uint64_t)live.size() + 64);
    const size_t half = P.N / 2 + 1;
    const size_t tiles = dexp_scan_tiles((uint32_t)half) + 1;
    hperm_status s = ensure_buf(c, B_DX_LEVELS, (size_t)L * P.W * 4);
    if (s) return s;
    s = ensure_buf(c, B_DX_OFFS, (size_t)L * P.N * 8);
    if (s) return s;
    s = ensure_buf(c, B_DX_AUX, half * 4 + 256 + 2 * half * 8 + 512 + tiles * 8 + 256 + sizeof(Misc) + 256 +
                                    (size_t)count * sizeof(ProbAcc) + 256 + (size_t)count * 4 + 256);
    if (s) return s;
    // deferred leaves are rare (orders above 16, or bounds beyond 64 bits): a first buffer of
    // 2^20 records, grown when a launch reports more
    P.wide_entries = (uint64_t)1 << 20;
    s = ensure_buf(c, B_SPLIT_WIDE, split_wide_bytes(P.wide_entries));
    if (s) return s;
    // (an arena re-layout may move any buffer: take every pointer after the last ensure_buf)
    P.levels = (uint32_t *)c->buf[B_DX_LEVELS].ptr;
    P.offs = (uint64_t *)c->buf[B_DX_OFFS].ptr;
    char *aux = (char *)c->buf[B_DX_AUX].ptr;
    auto take = [&aux](size_t bytes) {
        char *p = aux;
        aux += (bytes + 255) / 256 * 256;
        return (void *)p;
    };
    P.keys = (uint32_t *)take(half * 4);
    P.packed = (uint64_t *)take(half * 8);
    P.place = (uint64_t *)take(half * 8);
    P.tiles = (uint64_t *)take(tiles * 8);
    P.misc = (Misc *)take(sizeof(Misc));
    P.probs = (ProbAcc *)take((size_t)count * sizeof(ProbAcc));
    uint32_t *modps = (uint32_t *)take((size_t)count * 4);
    P.wide = c->buf[B_SPLIT_WIDE].ptr;
    P.maxw.assign((size_t)L, 0);
    P.maxw[(size_t)L - 1] = maxroot;
    c->resident_jobs = 0;   // the arena's layout may have moved the job table
    c->resident_list = 0;
    const double t0 = now_s();
    s = run.hip(hipMemcpyAsync(run.level(n), roots.data(), roots.size() * 4, hipMemcpyHostToDevice, c->stream),
                "upload roots");
    if (!s)
        s = run.hip(hipMemcpyAsync(run.offs(n), root_off.data(), root_off.size() * 8, hipMemcpyHostToDevice, c->stream),
                    "upload root offsets");
    if (!s && moduli) {
        s = run.hip(hipMemcpyAsync(modps, moduli->data(), (size_t)count * 4, hipMemcpyHostToDevice, c->stream),
                    "upload primes");
        P.modps = modps;
    }
    if (!s) s = run.hip(launch_fill_u64(&P.misc->grand, 3, 0ull, c->stream), "clear flags");
    if (!s) s = run.process(n, 0, live.size());
    if (!s) {   // the range flag of writes after the last continuation launch
        unsigned long long flags = 0;
        s = run.hip(hipMemcpyAsync(&flags, &P.misc->flags, 8, hipMemcpyDeviceToHost, c->stream), "download flags");
        if (!s) s = run.hip(hipStreamSynchronize(c->stream), "device expansion");
        if (!s && (flags & 1)) s = run.fail(HPERM_E_RANGE, "an expanded entry reached 2^22 or a row sum 2^24");
    }
    run.st.total_s = now_s() - t0;
    if (s) return set_error(c, s, run.err);
    if (sample) sample->complete = !run.stopped;
    if (moduli) {   // the sums of residues, reduced
        for (size_t k = 0; k < run.total.size(); ++k) {
            U512 &v = run.total[k];
            const uint64_t r = mod_u512(v, (*moduli)[k]);
            v = U512();
            v.w[0] = r;
        }
    } else if (!run.stopped) {
        for (int k : live)
            if (run.total[(size_t)k].bits() > (int)std::ceil(bounds[(size_t)k]) + 1)
                return set_error(c, HPERM_E_INTERNAL, "device expansion: a result exceeds its proven bound");
    }
    *out = run.total;
    if (stats) *stats = run.st;
    return HPERM_OK;
}

uint32_t residue_prime_limit(int n) {
    return (uint32_t)std::min<uint64_t>(1u << 18, ((1u << 24) - 1) / (uint64_t)std::max(n, 1) + 1);
}

double residue_bound_bits(const CsrView &a) {
    const int n = a.n;
    std::vector<double> cs((size_t)n, 0.0);
    double rb = 0.0, cb = 0.0;
    for (int i = 0; i < n; ++i) {
        double rs = 0.0;
        for (int32_t e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) {
            rs += a.val[e];
            cs[(size_t)a.col_idx[e]] += a.val[e];
        }
        if (rs == 0.0) return 0.0;
        rb += std::log2(rs);
    }
    for (int j = 0; j < n; ++j) {
        if (cs[(size_t)j] == 0.0) return 0.0;
        cb += std::log2(cs[(size_t)j]);
    }
    return std::min(rb, cb) * (1.0 + 1e-12);   // the sums' rounding
}

hperm_status device_expand_residues(Dev *c, const std::vector<CsrView> &probs, int T, int t, int s_leaf,
                                    size_t budget_bytes, std::vector<U512> *out, DexpStats *stats, int *nprimes) {
    out->assign(probs.size(), U512());
    if (probs.empty()) return HPERM_OK;
    const int n = probs[0].n;
    // the largest proven bound over the problems
    double bits = 0.0;
    for (const CsrView &a : probs) {
        if (a.n != n) return set_error(c, HPERM_E_INVALID, "residue evaluation: problems of one order");
        bits = std::max(bits, residue_bound_bits(a));
    }
    const std::vector<uint32_t> primes = residue_primes(residue_prime_limit(n), bits);
    double cover = 0.0;
    for (uint32_t q : primes) cover += std::log2((double)q);
    if (primes.empty() || cover > 511.0)
        return set_error(c, HPERM_E_RANGE, "residue evaluation: the permanent bound exceeds 2^500");
    const size_t K = primes.size() - 1, P = primes.size();
    // one device pass: every problem once per prime (problem k under prime j at j * count + k)
    std::vector<CsrView> all_probs;
    std::vector<uint32_t> moduli;
    for (size_t j = 0; j < P; ++j)
        for (const CsrView &a : probs) {
            all_probs.push_back(a);
            moduli.push_back(primes[j]);
        }
    std::vector<U512> tot;
    DexpStats all;
    const hperm_status s = device_expand_group(c, all_probs, T, t, s_leaf, budget_bytes, &tot, &all, nullptr, &moduli);
    if (s) return s;
    std::vector<uint64_t> r(probs.size() * P);
    for (size_t j = 0; j < P; ++j)
        for (size_t k = 0; k < probs.size(); ++k) r[k * P + j] = tot[j * probs.size() + k].w[0];
    const std::vector<uint32_t> base(primes.begin(), primes.begin() + (long)K);
    for (size_t k = 0; k < probs.size(); ++k) {
        const uint64_t *rk = r.data() + k * P;
        (*out)[k] = crt_garner(base, rk);
        if (mod_u512((*out)[k], primes[K]) != rk[K])
            return set_error(c, HPERM_E_INTERNAL, "residue evaluation: the check prime disagrees");
    }
    if (stats) *stats = all;
    if (nprimes) *nprimes = (int)P;
    return HPERM_OK;
}

hperm_status device_expand_problem(Dev *c, const CsrView &a, int T, int t, int s_leaf, size_t budget_bytes, U512 *out,
                                   DexpStats *stats, DexpSample *sample) {
    std::vector<U512> v;
    const hperm_status s = device_expand_group(c, std::vector<CsrView>{a}, T, t, s_leaf, budget_bytes, &v, stats, sample);
    if (s) return s;
    *out = v[0];
    return HPERM_OK;
}

}  // namespace hp
