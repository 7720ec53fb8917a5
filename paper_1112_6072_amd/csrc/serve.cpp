// Serving loop of libhperm: continuous batching of permanent requests.
//
// Requests are admitted while fewer than max_requests are live. Expansion workers expand
// admitted requests on the host (expansion (2), as in the blocking calls). A dispatcher packs
// every expanded request, oldest first, into one batch while the batch's device buffers fit
// in a free slice of the serving arena (admission by device memory), and runs the batch's
// jobs (estimate, one queue over all of the batch's jobs, persistent R-NW, recombination) on
// one of two streams, so a new batch starts while the previous one still runs. A completion
// thread finishes batches in launch order and delivers each request's exact result.
//
// Requests the device expansion takes (order above its job order, bound below 2^102) skip the
// host expansion: a device lane runs them, with the other waiting requests of the same order,
// by the device expansion on a stream of its own, so they overlap the batches. Requests the
// host expansion refuses for range (an expanded entry past 2^22, or the 2^180 bound) go to the
// device lane too when their order exceeds the device expansion's: it evaluates them exactly by
// residues (one device pass per prime, the Chinese remainder theorem). With a work limit, a
// request whose estimated GPU time (Knuth's estimate of its expansion tree, rated at the
// device path's measured leaf and subset-term rates, times twice the primes by residues)
// exceeds the limit is refused.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include <cmath>

#include "ctx.h"
#include "expand.h"
#include "kernels.h"

namespace hp {

namespace {

struct Request {
    uint64_t ticket = 0;
    int n = 0;
    std::vector<int32_t> rp, ci;
    std::vector<uint32_t> val;
    enum State { QUEUED, EXPANDING, READY, RUNNING, DONE } state = QUEUED;
    bool cancelled = false;
    hperm_jobs jobs;
    size_t bytes = 0;   // device bytes of this request's share of a batch
    uint64_t wide = 0;  // bound on its deferred wide leaves (device H_per)
    bool device = false;   // run by the device lane
    bool residues = false; // ... by residues (the exact paths refuse it for range)
    hperm_result result{};
    hperm_status status = HPERM_OK;
    std::string err;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

struct Batch {
    std::vector<Request *> reqs;
    hperm_jobs merged;
    int slot = 0;                // pipeline slot (stream and staging) it runs on
    size_t off = 0, bytes = 0;   // arena slice
    hperm_status status = HPERM_OK;
    std::string err;
};

// Device bytes of one batch part: the buffers of the pipeline for nd jobs, `words` data words
// and np problems, each buffer rounded up to 256 bytes (with split_order, also the device
// H_per counters and its record buffer for `wide` leaves above order 16).
size_t part_bytes(size_t nd, size_t words, size_t np, bool split, uint64_t wide) {
    auto al = [](size_t x) { return (std::max<size_t>(x, 1) + 255) / 256 * 256; };
    size_t b = al(nd * sizeof(JobDesc)) + al((words + 64) * 4) + al(nd * 4) /*bounds*/ + al(nd * 4) /*keys*/ +
               al(nd * 4) /*list*/ +
               al(nd * 4) /*queue*/ + al(nd * 8) /*items*/ + al(nd * sizeof(JobAcc)) + al(64 * 8) /*heads*/ +
               al(np * sizeof(ProbAcc)) + 2048;
    if (split) b += al(8 * 8) + al(split_wide_bytes(split_wide_capacity(wide, nd)));
    return b;
}

}  // namespace

struct Serving {
    hperm_ctx *ctx = nullptr;
    int max_requests = 0;
    void *arena = nullptr;
    size_t arena_bytes = 0;
    std::vector<std::pair<size_t, size_t>> free_list;   // (offset, size), sorted by offset
    // Two pipeline slots, each with its own stream, events and pinned staging: a batch is
    // enqueued on one while the batch before it still runs on the other. Batches complete in
    // launch order and at most two are in flight, so a slot is free again when its previous
    // batch has been completed.
    hipStream_t streams[2] = {nullptr, nullptr};
    Dev devs[2];
    int next_slot = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::deque<Request *> pending, ready, dev_ready;
    hipStream_t dev_stream = nullptr;   // the device lane's stream and buffers
    Dev devx;
    std::thread dev_lane;
    std::deque<std::unique_ptr<Batch>> inflight;
    uint64_t next_ticket = 1;
    bool stopping = false;
    bool dispatcher_done = false;
    std::vector<std::thread> workers;
    std::thread dispatcher, completer;

    bool alloc(size_t bytes, size_t *off) {
        for (size_t k = 0; k < free_list.size(); ++k)
            if (free_list[k].second >= bytes) {
                *off = free_list[k].first;
                free_list[k].first += bytes;
                free_list[k].second -= bytes;
                if (!free_list[k].second) free_list.erase(free_list.begin() + k);
                return true;
            }
        return false;
    }
    void release(size_t off, size_t bytes) {
        free_list.emplace_back(off, bytes);
        std::sort(free_list.begin(), free_list.end());
        std::vector<std::pair<size_t, size_t>> merged;
        for (auto &b : free_list) {
            if (!merged.empty() && merged.back().first + merged.back().second == b.first)
                merged.back().second += b.second;
            else
                merged.push_back(b);
        }
        free_list.swap(merged);
    }

    void expand_loop() {
        for (;;) {
            Request *r;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stopping || !pending.empty(); });
                if (stopping) return;
                r = pending.front();
                pending.pop_front();
                r->state = Request::EXPANDING;
            }
            const CsrView view{r->n, r->rp.data(), r->ci.data(), r->val.data()};
            double est_ms = 0.0;   // the work estimate (0 without a limit)
            if (ctx->opts.serve_limit_ms > 0 && r->n > 0) {
                // admission by work: Knuth's estimate of the tree, rated at about 5 ns per leaf
                // of the device continuation and 0.5 ns per R-NW subset-term
                const hperm_opts &o = ctx->opts;
                const int t = split_in_effect(o) > 0 ? split_in_effect(o) : o.m_cut;
                const int T = device_in_effect(o) > 0 ? device_in_effect(o) : o.m_cut;
                std::vector<double> nodes((size_t)r->n + 1), leaves((size_t)r->n + 1);
                const int rc = estimate_tree(view, std::max(T, t), t, o.s_leaf, 64, r->ticket, nodes.data(),
                                             leaves.data());
                double ms = 0.0;
                for (int p = 0; p <= r->n; ++p) ms += leaves[(size_t)p] * (5e-6 + std::ldexp(5e-10, p - 1));
                if (rc == 0) est_ms = ms;
                if (rc == 0 && ms > o.serve_limit_ms) {
                    std::lock_guard<std::mutex> lk(mu);
                    r->status = HPERM_E_TOOBIG;
                    r->err = "estimated work " + std::to_string((long long)ms) + " ms exceeds the serving limit of " +
                             std::to_string(o.serve_limit_ms) + " ms";
                    r->state = Request::DONE;
                    r->t_done = now_s();
                    cv.notify_all();
                    continue;
                }
            }
            if (device_path(ctx->opts, view)) {   // the device lane takes it
                std::lock_guard<std::mutex> lk(mu);
                if (r->cancelled) {
                    r->state = Request::DONE;
                    r->t_done = now_s();
                } else {
                    r->device = true;
                    r->state = Request::READY;
                    dev_ready.push_back(r);
                }
                cv.notify_all();
                continue;
            }
            ExpandParams prm = expand_params(ctx->opts);
            if (prm.threads == 0) prm.threads = 2;
            std::vector<CsrView> probs{view};
            std::string err;
            const int rc = expand_problems(probs, prm, &r->jobs.tab, &err);
            std::lock_guard<std::mutex> lk(mu);
            if (r->cancelled) {   // cancelled while expanding: no GPU work
                r->jobs.tab = JobTable();
                r->state = Request::DONE;
                r->t_done = now_s();
            } else if (rc == -2 && residue_path(ctx->opts, r->n)) {
                // out of the exact paths' range: the device lane evaluates it by residues, one
                // device pass per prime (each rated at twice the exact pass's work)
                r->jobs.tab = JobTable();
                const size_t np = residue_primes(residue_prime_limit(r->n), residue_bound_bits(view)).size();
                const double ms = est_ms * 2.0 * (double)np;
                if (ctx->opts.serve_limit_ms > 0 && ms > ctx->opts.serve_limit_ms) {
                    r->status = HPERM_E_TOOBIG;
                    r->err = "estimated work " + std::to_string((long long)ms) + " ms by residues (" +
                             std::to_string(np) + " primes) exceeds the serving limit of " +
                             std::to_string(ctx->opts.serve_limit_ms) + " ms";
                    r->state = Request::DONE;
                    r->t_done = now_s();
                } else {
                    r->device = true;
                    r->residues = true;
                    r->state = Request::READY;
                    dev_ready.push_back(r);
                }
            } else if (rc) {
                r->status = rc == -2 ? HPERM_E_RANGE : rc == -3 ? HPERM_E_NOMEM : HPERM_E_INVALID;
                r->err = err;
                r->state = Request::DONE;
                r->t_done = now_s();
            } else if (r->jobs.tab.desc.empty()) {
                // no GPU work: n = 0 or a zero line
                r->result = hperm_result{};
                const uint64_t v = r->jobs.tab.direct_valid[0] ? r->jobs.tab.direct_value[0] : 0;
                r->result.limb[0] = v;
                r->result.nlimb = v ? 1 : 0;
                r->state = Request::DONE;
                r->t_done = now_s();
            } else {
                const auto &t = r->jobs.tab;
                r->wide = split_wide_total(t.desc, ctx->opts);
                r->bytes = part_bytes(t.desc.size(), t.data.size(), 1, ctx->opts.split_order != 0 && ctx->opts.s_leaf <= 5,
                                      r->wide);
                if (r->bytes > arena_bytes) {
                    r->status = HPERM_E_NOMEM;
                    r->err = "request needs " + std::to_string(r->bytes) + " device bytes; the serving arena holds " +
                             std::to_string(arena_bytes);
                    r->state = Request::DONE;
                    r->t_done = now_s();
                } else {
                    r->state = Request::READY;
                    ready.push_back(r);
                }
            }
            cv.notify_all();
        }
    }

    void dispatch_loop() {
        for (;;) {
            std::unique_ptr<Batch> b(new Batch());
            {
                std::unique_lock<std::mutex> lk(mu);
                size_t off = 0;
                cv.wait(lk, [&] {
                    if (stopping) return true;
                    if (ready.empty() || inflight.size() >= 2) return false;
                    return alloc_probe(ready.front()->bytes);
                });
                if (stopping) break;
                // take the oldest ready requests while the batch fits a free arena slice
                size_t need = 0, nd = 0, words = 0;
                uint64_t wide = 0;
                std::vector<Request *> take;
                size_t largest = 0;
                for (auto &f : free_list) largest = std::max(largest, f.second);
                for (Request *r : ready) {
                    const auto &t = r->jobs.tab;
                    const size_t cand = part_bytes(nd + t.desc.size(), words + t.data.size(), take.size() + 1,
                                                   ctx->opts.split_order != 0 && ctx->opts.s_leaf <= 5, wide + r->wide);
                    if (cand > largest) break;
                    take.push_back(r);
                    nd += t.desc.size();
                    words += t.data.size();
                    wide += r->wide;
                    need = cand;
                }
                if (take.empty()) continue;
                if (!alloc(need, &off)) continue;
                ready.erase(ready.begin(), ready.begin() + take.size());
                const double t = now_s();
                for (Request *r : take) {
                    r->state = Request::RUNNING;
                    r->t_admit = t;
                }
                b->reqs = take;
                b->off = off;
                b->bytes = need;
                b->slot = next_slot;
                next_slot ^= 1;
            }
            // merge the requests' job tables: problem k of the batch is request k
            JobTable &m = b->merged.tab;
            if (b->reqs.size() == 1) {
                m = std::move(b->reqs[0]->jobs.tab);
            } else {
                for (size_t k = 0; k < b->reqs.size(); ++k) {
                    JobTable &t = b->reqs[k]->jobs.tab;
                    m.data.resize(hp_align_words(m.data.size()));
                    const uint32_t shift = (uint32_t)(m.data.size() / HP_DATA_ALIGN);
                    for (JobDesc d : t.desc) {
                        d.data_off += shift;
                        d.problem = (uint32_t)k;
                        m.desc.push_back(d);
                    }
                    m.data.insert(m.data.end(), t.data.begin(), t.data.end());
                    m.log2_bound.insert(m.log2_bound.end(), t.log2_bound.begin(), t.log2_bound.end());
                    m.direct_valid.push_back(0);
                    m.direct_value.push_back(0);
                    m.problem_log2_bound.push_back(t.problem_log2_bound[0]);
                    t = JobTable();
                }
                m.n_problems = (int)b->reqs.size();
            }
            b->merged.id = next_jobs_id();
            Dev &d = devs[b->slot];
            for (auto &buf : d.buf) buf = DevBuf();   // slices of the previous batch's arena block
            d.arena = (char *)arena + b->off;
            d.arena_bytes = b->bytes;
            d.resident_jobs = 0;
            d.opts = ctx->opts;
            d.tune = ctx->dev.tune;
            d.opts.time_jobs = 0;   // job timing is for the blocking stage calls only
            d.opts.use_graphs = 0;  // every batch is a new job table: nothing to replay
            hperm_status s = HPERM_OK;
            if (d.opts.order == HPERM_ORDER_ESTIMATE || d.opts.order == HPERM_ORDER_EXACT_COST)
                s = estimate_jobs(&d, &b->merged, d.opts.trials, d.opts.seed);
            if (!s) s = run_enqueue(&d, &b->merged, d.opts.order, 1, false);
            b->status = s;
            if (s) b->err = d.last_error;
            std::lock_guard<std::mutex> lk(mu);
            inflight.push_back(std::move(b));
            cv.notify_all();
        }
        std::lock_guard<std::mutex> lk(mu);
        dispatcher_done = true;
        cv.notify_all();
    }

    // The device lane: the oldest waiting request's order and every waiting request of that
    // order (and of its kind: exact, or by residues), expanded on the device together. An exact
    // group refused for range (an expanded entry past 2^22) is evaluated again by residues.
    void device_loop() {
        const size_t budget = (size_t)(ctx->opts.device_expand_mib > 0 ? ctx->opts.device_expand_mib : 8192) << 20;
        for (;;) {
            std::vector<Request *> grp;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stopping || !dev_ready.empty(); });
                if (stopping) return;
                const int n = dev_ready.front()->n;
                const bool byres = dev_ready.front()->residues;
                for (auto it = dev_ready.begin(); it != dev_ready.end();) {
                    if ((*it)->n == n && (*it)->residues == byres) {
                        grp.push_back(*it);
                        it = dev_ready.erase(it);
                    } else {
                        ++it;
                    }
                }
                const double t = now_s();
                for (Request *r : grp) {
                    r->state = Request::RUNNING;
                    r->t_admit = t;
                }
            }
            std::vector<CsrView> views;
            for (Request *r : grp) views.push_back(CsrView{r->n, r->rp.data(), r->ci.data(), r->val.data()});
            devx.opts = ctx->opts;
            devx.tune = ctx->dev.tune;
            std::vector<U512> totals;
            DexpStats st;
            bool byres = grp[0]->residues;
            hperm_status s = HPERM_OK;
            if (!byres) {
                s = device_expand_group(&devx, views, device_in_effect(devx.opts), split_in_effect(devx.opts),
                                        devx.opts.s_leaf, budget, &totals, &st);
                byres = s == HPERM_E_RANGE && residue_path(devx.opts, grp[0]->n);
            }
            if (byres)
                s = device_expand_residues(&devx, views, device_in_effect(devx.opts), split_in_effect(devx.opts),
                                           devx.opts.s_leaf, budget, &totals, &st, nullptr);
            std::lock_guard<std::mutex> lk(mu);
            const double t = now_s();
            for (size_t k = 0; k < grp.size(); ++k) {
                Request *r = grp[k];
                r->status = s;
                if (s) {
                    r->err = devx.last_error;
                } else {
                    r->result = hperm_result{};
                    fill_result(totals[k], &r->result);
                    r->result.n_jobs = (int32_t)std::min<uint64_t>(st.jobs, 0x7fffffff);
                    r->result.max_m = device_in_effect(devx.opts);
                    r->result.arith_mask = 1 << (byres ? HPERM_ARITH_RES : HPERM_ARITH_W64);
                    r->result.subset_terms = st.leaf_terms;
                    r->result.t_rnw_s = st.split_s;
                }
                r->state = Request::DONE;
                r->t_done = t;
            }
            cv.notify_all();
        }
    }

    // Whether some free slice holds `bytes` (caller holds mu).
    bool alloc_probe(size_t bytes) const {
        for (auto &f : free_list)
            if (f.second >= bytes) return true;
        return false;
    }

    void complete_loop() {
        for (;;) {
            Batch *b;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return !inflight.empty() || (stopping && dispatcher_done); });
                if (inflight.empty()) return;
                b = inflight.front().get();
            }
            std::vector<hperm_result> totals(b->reqs.size());
            double t_rnw = 0.0;
            hperm_status s = b->status;
            Dev &d = devs[b->slot];
            if (!s) {
                s = run_finish(&d, &b->merged, nullptr, totals.data(), &t_rnw);
                if (s) b->err = d.last_error;
            }
            (void)hipStreamSynchronize(d.stream);   // nothing of the batch may still use its slice
            std::lock_guard<std::mutex> lk(mu);
            const double t = now_s();
            for (size_t k = 0; k < b->reqs.size(); ++k) {
                Request *r = b->reqs[k];
                r->status = s;
                r->err = b->err;
                if (!s) r->result = totals[k];
                r->result.t_rnw_s = t_rnw;
                r->state = Request::DONE;
                r->t_done = t;
            }
            release(b->off, b->bytes);
            inflight.pop_front();
            cv.notify_all();
        }
    }

    void finish_result(Request *r, hperm_result *out) {
        if (out) {
            *out = r->result;
            out->t_expand_s = r->t_admit > 0 ? r->t_admit - r->t_submit : 0.0;
            out->t_total_s = r->t_done - r->t_submit;
        }
    }
};

void serve_shutdown(hperm_ctx *c) {
    Serving *sv = c->serving;
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
        sv->cv.notify_all();
    }
    for (auto &t : sv->workers) t.join();
    sv->dispatcher.join();
    sv->completer.join();
    if (sv->dev_lane.joinable()) sv->dev_lane.join();
    for (Dev &d : sv->devs) dev_release(&d);
    dev_release(&sv->devx);
    if (sv->dev_stream) (void)hipStreamDestroy(sv->dev_stream);
    for (hipStream_t s : sv->streams)
        if (s) (void)hipStreamDestroy(s);
    if (sv->arena) (void)hipFree(sv->arena);
    delete sv;
    c->serving = nullptr;
}

}  // namespace hp

using namespace hp;

extern "C" {

hperm_status hperm_serve_start(hperm_ctx *c, int32_t max_requests, size_t arena_bytes) {
    if (!c) return HPERM_E_INVALID;
    if (c->host_only) return set_error(c, HPERM_E_DEVICE, "host-only context");
    if (c->serving) return set_error(c, HPERM_E_INVALID, "already serving");
    if (max_requests < 1 || max_requests > 65536)
        return set_error(c, HPERM_E_INVALID, "max_requests must be in [1, 65536]");
    if (arena_bytes == 0) arena_bytes = (size_t)1 << 31;
    Serving *sv = new (std::nothrow) Serving();
    if (!sv) return HPERM_E_NOMEM;
    sv->ctx = c;
    sv->max_requests = max_requests;
    if (hipMalloc(&sv->arena, arena_bytes) != hipSuccess) {
        delete sv;
        return set_error(c, HPERM_E_NOMEM, "serving arena allocation failed");
    }
    sv->arena_bytes = arena_bytes;
    sv->free_list.emplace_back(0, arena_bytes);
    for (int k = 0; k < 2; ++k) {
        if (hipStreamCreateWithFlags(&sv->streams[k], hipStreamNonBlocking) != hipSuccess) {
            for (int q = 0; q < k; ++q) (void)hipStreamDestroy(sv->streams[q]);
            (void)hipFree(sv->arena);
            delete sv;
            return set_error(c, HPERM_E_DEVICE, "stream creation failed");
        }
        sv->devs[k].stream = sv->streams[k];
    }
    if (hipStreamCreateWithFlags(&sv->dev_stream, hipStreamNonBlocking) != hipSuccess) {
        for (hipStream_t st : sv->streams) (void)hipStreamDestroy(st);
        (void)hipFree(sv->arena);
        delete sv;
        return set_error(c, HPERM_E_DEVICE, "stream creation failed");
    }
    sv->devx.stream = sv->dev_stream;
    sv->devx.last_error.reserve(256);
    c->serving = sv;
    for (int k = 0; k < 4; ++k) sv->workers.emplace_back([sv] { sv->expand_loop(); });
    sv->dev_lane = std::thread([sv] { sv->device_loop(); });
    sv->dispatcher = std::thread([sv] { sv->dispatch_loop(); });
    sv->completer = std::thread([sv] { sv->complete_loop(); });
    return HPERM_OK;
}

hperm_status hperm_serve_stop(hperm_ctx *c) {
    if (!c) return HPERM_E_INVALID;
    if (!c->serving) return set_error(c, HPERM_E_INVALID, "not serving");
    serve_shutdown(c);
    return HPERM_OK;
}

hperm_status hperm_submit(hperm_ctx *c, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                          const uint32_t *val, uint64_t *ticket) {
    if (!c || !ticket) return HPERM_E_INVALID;
    Serving *sv = c->serving;
    if (!sv) return HPERM_E_INVALID;
    const std::string why = validate_csr(CsrView{n, row_ptr, col_idx, val});
    if (!why.empty()) {
        std::lock_guard<std::mutex> lk(sv->mu);
        c->dev.last_error = why;
        return HPERM_E_INVALID;
    }
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return HPERM_E_NOMEM;
    r->n = n;
    const int nnz = n > 0 ? row_ptr[n] : 0;
    if (n > 0) r->rp.assign(row_ptr, row_ptr + n + 1);
    else r->rp.assign(1, 0);
    if (nnz > 0) {
        r->ci.assign(col_idx, col_idx + nnz);
        r->val.assign(val, val + nnz);
    }
    r->ci.push_back(0);
    r->val.push_back(0);
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stopping) return HPERM_E_INVALID;
    if ((int)sv->reqs.size() >= sv->max_requests) {
        c->dev.last_error = "all request slots are in use";
        return HPERM_E_BUSY;
    }
    r->ticket = sv->next_ticket++;
    r->t_submit = now_s();
    *ticket = r->ticket;
    sv->pending.push_back(r.get());
    sv->reqs.emplace(r->ticket, std::move(r));
    sv->cv.notify_all();
    return HPERM_OK;
}

// Caller holds sv->mu.
static hperm_status take_result(hperm_ctx *c, uint64_t ticket, hperm_result *out) {
    Serving *sv = c->serving;
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) {
        c->dev.last_error = "unknown ticket";
        return HPERM_E_INVALID;
    }
    Request *r = it->second.get();
    if (r->state != Request::DONE) return HPERM_NOT_READY;
    hperm_status s = r->cancelled ? HPERM_E_CANCELLED : r->status;
    if (!s) sv->finish_result(r, out);
    else c->dev.last_error = r->cancelled ? std::string("request cancelled") : r->err;
    sv->reqs.erase(it);
    sv->cv.notify_all();
    return s;
}

hperm_status hperm_poll(hperm_ctx *c, uint64_t ticket, hperm_result *out) {
    if (!c || !c->serving) return HPERM_E_INVALID;
    std::lock_guard<std::mutex> lk(c->serving->mu);
    return take_result(c, ticket, out);
}

hperm_status hperm_wait(hperm_ctx *c, uint64_t ticket, double timeout_s, hperm_result *out) {
    if (!c || !c->serving) return HPERM_E_INVALID;
    Serving *sv = c->serving;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto done = [&] {
        auto it = sv->reqs.find(ticket);
        return it == sv->reqs.end() || it->second->state == Request::DONE;
    };
    if (timeout_s < 0) {
        sv->cv.wait(lk, done);
    } else if (!sv->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
        return HPERM_E_TIMEOUT;
    }
    return take_result(c, ticket, out);
}

hperm_status hperm_cancel(hperm_ctx *c, uint64_t ticket) {
    if (!c || !c->serving) return HPERM_E_INVALID;
    Serving *sv = c->serving;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return HPERM_E_INVALID;
    Request *r = it->second.get();
    r->cancelled = true;
    if (r->state == Request::QUEUED) {
        sv->pending.erase(std::find(sv->pending.begin(), sv->pending.end(), r));
        r->state = Request::DONE;
        r->t_done = now_s();
    } else if (r->state == Request::READY) {
        if (r->device) sv->dev_ready.erase(std::find(sv->dev_ready.begin(), sv->dev_ready.end(), r));
        else sv->ready.erase(std::find(sv->ready.begin(), sv->ready.end(), r));
        r->state = Request::DONE;
        r->t_done = now_s();
    }
    sv->cv.notify_all();
    return HPERM_OK;
}

}  // extern "C"
