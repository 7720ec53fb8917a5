// Autotuner of the persistent R-NW launches: per launch group of a job table (ring, order
// bucket, walk variant) it times the group's kernel on a sample of its jobs for candidate lane
// chunks (Gray indices per lane, hence work items, i.e. waves, per job) and persistent grids,
// keeps the fastest pair in the context's tuning table (used by every later persistent run on
// the context) and can cache the table as JSON keyed by the GPU architecture.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"
#include "kernels.h"

using namespace hp;

namespace {

const int kDeltas[] = {-3, -2, -1, 0, 1};
const int kGrids[] = {100, 75, 50};
const uint64_t kSampleTerms = 1ull << 33;   // about 4 ms of the mod-2^64 walk per trial

int tuned_chunk_of(int m, int c0, int delta, int cmin) {   // as the queue builder applies it
    int c = c0 + delta;
    if (c > 12) c = 12;
    if (c > m - 1) c = std::max(0, m - 1);
    if (c < cmin) c = std::min(cmin, std::max(0, m - 1));
    if (c < m - 32) c = m - 32;
    return c;
}

uint64_t items_for(int m, int c) {
    const int e = m - 1 - 6 - c;
    return e > 0 ? (1ull << e) : 1ull;
}

std::string arch_name(int device) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t k = a.find(':');
    return k == std::string::npos ? a : a.substr(0, k);
}

// The cache file: {"<arch>": {"<ring>/<bucket>/<variant>": [chunk_delta, grid_pct], ...}, ...}
// (this writer's own format; anything else is ignored).
struct CacheEntry {
    std::string arch;
    int ring, bucket, variant, delta, grid;
};

std::vector<CacheEntry> read_cache(const char *path) {
    std::vector<CacheEntry> out;
    FILE *f = fopen(path, "rb");
    if (!f) return out;
    std::string txt;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, k);
    fclose(f);
    size_t i = 0;
    auto skip = [&]() {
        while (i < txt.size() && strchr(" \t\r\n,:", txt[i])) ++i;
    };
    auto str = [&](std::string *s) {
        skip();
        if (i >= txt.size() || txt[i] != '"') return false;
        const size_t e = txt.find('"', i + 1);
        if (e == std::string::npos) return false;
        *s = txt.substr(i + 1, e - i - 1);
        i = e + 1;
        return true;
    };
    skip();
    if (i >= txt.size() || txt[i] != '{') return out;
    ++i;
    for (;;) {
        std::string arch;
        if (!str(&arch)) break;
        skip();
        if (i >= txt.size() || txt[i] != '{') break;
        ++i;
        for (;;) {
            std::string key;
            if (!str(&key)) break;
            skip();
            int d = 0, g = 0, r = 0, b = 0, v = 0;
            if (sscanf(txt.c_str() + i, "[%d , %d]", &d, &g) != 2 && sscanf(txt.c_str() + i, "[%d,%d]", &d, &g) != 2) break;
            i = txt.find(']', i);
            if (i == std::string::npos) return out;
            ++i;
            if (sscanf(key.c_str(), "%d/%d/%d", &r, &b, &v) == 3) out.push_back(CacheEntry{arch, r, b, v, d, g});
        }
        skip();
        if (i < txt.size() && txt[i] == '}') ++i;
    }
    return out;
}

bool write_cache(const char *path, const std::vector<CacheEntry> &entries) {
    std::vector<std::string> archs;
    for (const auto &e : entries)
        if (std::find(archs.begin(), archs.end(), e.arch) == archs.end()) archs.push_back(e.arch);
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return false;
    fprintf(f, "{\n");
    for (size_t a = 0; a < archs.size(); ++a) {
        fprintf(f, "  \"%s\": {", archs[a].c_str());
        bool first = true;
        for (const auto &e : entries)
            if (e.arch == archs[a]) {
                fprintf(f, "%s\n    \"%d/%d/%d\": [%d, %d]", first ? "" : ",", e.ring, e.bucket, e.variant, e.delta, e.grid);
                first = false;
            }
        fprintf(f, "\n  }%s\n", a + 1 < archs.size() ? "," : "");
    }
    fprintf(f, "}\n");
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" hperm_status hperm_autotune(hperm_ctx *c, hperm_jobs *j, const char *cache_path, int32_t force,
                                       hperm_tune_entry *out, int32_t max, int32_t *n_out) {
    if (c && c->host_only) return set_error(c, HPERM_E_DEVICE, "host-only context");
    if (!c || max < 0 || (max > 0 && !out)) return HPERM_E_INVALID;
    if (c->serving) return set_error(c, HPERM_E_INVALID, "the context is serving");
    std::lock_guard<std::mutex> lk(c->call_mu);
    Dev *d = &c->dev;
    d->opts = c->opts;
    const std::string arch = arch_name(c->device);
    std::vector<CacheEntry> cache = cache_path ? read_cache(cache_path) : std::vector<CacheEntry>();
    std::vector<hperm_tune_entry> res;
    {   // cached entries of this architecture enter the table
        std::lock_guard<std::mutex> tl(d->tune->mu);
        bool any = false;
        for (const auto &e : cache)
            if (e.arch == arch) {
                TuneEntry te;
                te.chunk_delta = std::max(-12, std::min(12, e.delta));
                te.grid_pct = std::max(10, std::min(100, e.grid));
                const int key = tune_key(e.ring, e.bucket, e.variant);
                if (!force || !j) {
                    d->tune->e[key] = te;
                    any = true;
                }
            }
        if (any) d->tune->version++;
    }
    if (j && !j->tab.desc.empty()) {
        const size_t nd = j->tab.desc.size();
        hperm_status s = upload_jobs(d, j);
        if (s) return s;
        // the jobs' own chunks (before any tuning) and their groups
        if (j->chunk0.size() != nd) {
            j->chunk0.resize(nd);
            for (size_t k = 0; k < nd; ++k) j->chunk0[k] = j->tab.desc[k].chunk_log2;
        }
        std::map<int, std::vector<uint32_t>> groups;
        for (size_t k = 0; k < nd; ++k) {
            JobDesc d0 = j->tab.desc[k];
            d0.chunk_log2 = j->chunk0[k];
            if (d0.chunk_log2 == 0) continue;   // single-index lanes: nothing to tune
            groups[tune_key(d0.arith, bucket_of(d0.m), walk_variant(d0, d0.chunk_log2))].push_back((uint32_t)k);
        }
        if (!d->ev0) {
            s = hip_check(d, hipEventCreate(&d->ev0), "hipEventCreate");
            if (s) return s;
            s = hip_check(d, hipEventCreate(&d->ev1), "hipEventCreate");
            if (s) return s;
        }
        for (auto &gk : groups) {
            const int key = gk.first;
            const int ring = tune_key_ring(key), bucket = tune_key_bucket(key), variant = tune_key_variant(key);
            bool cached = false;
            {
                std::lock_guard<std::mutex> tl(d->tune->mu);
                cached = d->tune->e.count(key) && !force;
            }
            if (cached) continue;
            // the sample: the group's first jobs (natural order) up to kSampleTerms subset-terms
            std::vector<uint32_t> sample;
            uint64_t terms = 0;
            for (uint32_t k : gk.second) {
                sample.push_back(k);
                terms += 1ull << (j->tab.desc[k].m - 1);
                if (terms >= kSampleTerms) break;
            }
            const size_t K = sample.size();
            s = ensure_buf(d, B_TUNE_DESC, K * sizeof(JobDesc));
            if (!s) s = ensure_buf(d, B_TUNE_QUEUE, K * 4 + K * 8 + 64);
            if (!s) s = ensure_buf(d, B_ACCS, K * sizeof(JobAcc));
            if (!s) s = ensure_buf(d, B_HEAD, 64 * 8);
            if (s) return s;
            if (d->resident_jobs != j->id) {   // an arena re-layout moved the table
                s = upload_jobs(d, j);
                if (s) return s;
            }
            std::vector<uint32_t> q(K);
            for (size_t k = 0; k < K; ++k) q[k] = (uint32_t)k;
            uint32_t *tq = (uint32_t *)d->buf[B_TUNE_QUEUE].ptr;
            uint64_t *ti = (uint64_t *)((char *)d->buf[B_TUNE_QUEUE].ptr + ((K * 4 + 63) / 64) * 64);
            s = hip_check(d, hipMemcpy(tq, q.data(), K * 4, hipMemcpyHostToDevice), "upload tuning queue");
            if (s) return s;
            double best_ms = 1e300, def_ms = 0.0;
            int best_delta = 0, best_grid = 100;
            std::vector<int> seen_chunks;
            for (int delta : kDeltas) {
                std::vector<JobDesc> td(K);
                std::vector<uint64_t> ie(K);
                uint64_t acc = 0;
                int sig = 0;
                for (size_t k = 0; k < K; ++k) {
                    td[k] = j->tab.desc[sample[k]];
                    // the four-step walks (variants 6, 7) need lane chunks of 4 steps at least
                    const int ch = tuned_chunk_of(td[k].m, j->chunk0[sample[k]], delta, variant >= 6 ? 2 : 1);
                    td[k].chunk_log2 = (uint8_t)ch;
                    if (k == 0) sig = ch;
                    ie[k] = acc += items_for(td[k].m, ch);
                }
                if (delta != 0 && std::find(seen_chunks.begin(), seen_chunks.end(), sig) != seen_chunks.end()) continue;
                seen_chunks.push_back(sig);
                s = hip_check(d, hipMemcpy(d->buf[B_TUNE_DESC].ptr, td.data(), K * sizeof(JobDesc), hipMemcpyHostToDevice),
                              "upload tuning descriptors");
                if (!s) s = hip_check(d, hipMemcpy(ti, ie.data(), K * 8, hipMemcpyHostToDevice), "upload tuning items");
                if (s) return s;
                int full = 0;
                s = hip_check(d, persistent_grid(ring, bucket, variant, &full), "persistent grid");
                if (s) return s;
                for (int gp : kGrids) {
                    double ms = 1e300;
                    for (int rep = 0; rep < 2; ++rep) {
                        s = hip_check(d, launch_fill_u64((unsigned long long *)d->buf[B_HEAD].ptr, 64, 0ull, d->stream),
                                      "clear heads");
                        if (!s)
                            s = hip_check(d, launch_fill_u64((unsigned long long *)d->buf[B_ACCS].ptr, K * 8, 0ull, d->stream),
                                          "clear accumulators");
                        if (!s) s = hip_check(d, hipEventRecord(d->ev0, d->stream), "event");
                        if (!s)
                            s = hip_check(d, launch_rnw_persistent(ring, bucket, variant, (const JobDesc *)d->buf[B_TUNE_DESC].ptr,
                                                                   (const uint32_t *)d->buf[B_DATA].ptr, tq, ti, (uint32_t)K, acc,
                                                                   (unsigned long long *)d->buf[B_HEAD].ptr,
                                                                   (JobAcc *)d->buf[B_ACCS].ptr, nullptr,
                                                                   std::max(1, full * gp / 100), d->stream),
                                          "tuning launch");
                        if (!s) s = hip_check(d, hipEventRecord(d->ev1, d->stream), "event");
                        if (!s) s = hip_check(d, hipStreamSynchronize(d->stream), "tuning launch");
                        if (s) return s;
                        float t = 0.0f;
                        (void)hipEventElapsedTime(&t, d->ev0, d->ev1);
                        ms = std::min(ms, (double)t);
                    }
                    if (delta == 0 && gp == 100) def_ms = ms;
                    if (ms < best_ms * 0.98 || (delta == 0 && gp == 100 && ms <= best_ms)) {
                        best_ms = ms;
                        best_delta = delta;
                        best_grid = gp;
                    }
                }
            }
            // keep the default unless a choice is at least 2 % faster
            if (best_ms > def_ms * 0.98) {
                best_ms = def_ms;
                best_delta = 0;
                best_grid = 100;
            }
            TuneEntry te;
            te.chunk_delta = best_delta;
            te.grid_pct = best_grid;
            te.ms_default = def_ms;
            te.ms_tuned = best_ms;
            {
                std::lock_guard<std::mutex> tl(d->tune->mu);
                d->tune->e[key] = te;
                d->tune->version++;
            }
            bool found = false;
            for (auto &e : cache)
                if (e.arch == arch && e.ring == ring && e.bucket == bucket && e.variant == variant) {
                    e.delta = best_delta;
                    e.grid = best_grid;
                    found = true;
                }
            if (!found) cache.push_back(CacheEntry{arch, ring, bucket, variant, best_delta, best_grid});
        }
        if (cache_path && !write_cache(cache_path, cache))
            return set_error(c, HPERM_E_INVALID, "cannot write the tuning cache");
    }
    {
        std::lock_guard<std::mutex> tl(d->tune->mu);
        for (const auto &kv : d->tune->e) {
            hperm_tune_entry e{};
            e.ring = tune_key_ring(kv.first);
            e.bucket = tune_key_bucket(kv.first);
            e.variant = tune_key_variant(kv.first);
            e.chunk_delta = kv.second.chunk_delta;
            e.grid_pct = kv.second.grid_pct;
            e.from_cache = kv.second.ms_default == 0.0;
            e.ms_default = kv.second.ms_default;
            e.ms_tuned = kv.second.ms_tuned;
            res.push_back(e);
        }
    }
    const int32_t k = (int32_t)std::min<size_t>(res.size(), (size_t)max);
    for (int32_t q = 0; q < k; ++q) out[q] = res[(size_t)q];
    if (n_out) *n_out = (int32_t)res.size();
    return HPERM_OK;
}

extern "C" hperm_status hperm_tune_clear(hperm_ctx *c) {
    if (!c) return HPERM_E_INVALID;
    if (c->host_only) return set_error(c, HPERM_E_DEVICE, "host-only context");
    std::lock_guard<std::mutex> tl(c->dev.tune->mu);
    c->dev.tune->e.clear();
    c->dev.tune->version++;
    return HPERM_OK;
}
