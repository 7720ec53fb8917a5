// Context and job-table objects behind the C ABI of libhperm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hperm.h"
#include "bigint.h"
#include "expand.h"

namespace hp {

// A device buffer, either from hipMalloc (grown on demand) or a slice of the caller's arena.
struct DevBuf {
    void *ptr = nullptr;
    size_t cap = 0;
    bool owned = false;
};

enum BufId { B_DESC, B_DESC_PLAIN, B_DATA, B_BOUND, B_KEYS, B_LIST, B_QUEUE, B_ITEMS, B_ACCS, B_HEAD, B_PROB, B_CYCLES,
             B_SPLIT, B_SPLIT_WIDE, B_DX_LEVELS, B_DX_OFFS, B_DX_AUX, B_TUNE_DESC, B_TUNE_QUEUE, B_COUNT };

struct Serving;   // serve.cpp

// Tuned launch settings of the persistent R-NW kernels, per launch group (ring, order bucket,
// walk variant): the lane chunk as an offset from each job's default chunk (which sets the
// Gray indices per lane and so the work items, i.e. the waves, of a job) and the persistent
// grid as a percentage of the resident one.
struct TuneEntry {
    int chunk_delta = 0;
    int grid_pct = 100;
    double ms_default = 0.0, ms_tuned = 0.0;   // the timed trials that chose it (0: from a cache)
};
struct TuneTable {
    std::mutex mu;
    std::map<int, TuneEntry> e;   // key: tune_key(ring, bucket, variant)
    uint64_t version = 0;         // bumped on every change
};
inline int tune_key(int ring, int bucket, int variant) { return (ring * 8 + bucket) * 8 + variant; }
inline int tune_key_ring(int key) { return key / 64; }
inline int tune_key_bucket(int key) { return (key / 8) % 8; }
inline int tune_key_variant(int key) { return key % 8; }

}  // namespace hp

struct hperm_jobs {
    hp::JobTable tab;
    std::vector<float> keys;   // KKLLL keys, natural index
    std::vector<float> fbound; // proven log2 bounds of the jobs as floats rounded up
    bool has_keys = false;
    uint64_t id = 0;           // identity for device residency
    // The persistent queue's grouping, which does not depend on the job order: per job its
    // launch group and work items; per group its ring, order bucket, walk and totals (jobs,
    // items, subset-terms, algorithmic work). Filled on the first persistent run.
    struct QueueGroup {
        int ring, bucket, variant;
        size_t n;
        uint64_t items, terms;
        double mults, adds, updates;
        int mmax = 0;        // device H_per group: largest job order
        uint64_t wide = 0;   // ... and the bound on its deferred wide leaves
        double extra = 0.0;  // full-rate slots besides ring operations and row updates
    };
    // the estimator's job list (jobs grouped by its order buckets, natural order inside) and
    // the bucket offsets, also filled once
    std::vector<uint32_t> elist;
    std::vector<size_t> eoff;
    std::vector<uint8_t> qgroup;
    std::vector<uint64_t> qitems;
    std::vector<QueueGroup> qgroups;
    int qsplit = -1;   // split_order the launch groups were built for
    // per-job work cycles of the last timed persistent run (natural index)
    std::vector<uint64_t> cycles;
    bool has_cycles = false;
    // the lane chunks the expansion chose (restored when the tuning changes) and the tuning
    // version the table's chunks follow
    std::vector<uint8_t> chunk0;
    uint64_t tune_version = 0;
    const void *tune_table = nullptr;
};

namespace hp {

// What a captured run graph depends on (api.cpp, graph_key).
struct GraphKey {
    uint64_t jobs_id = 0;
    size_t nd = 0;
    int np = 0;
    void *bufs[B_COUNT] = {};
    int split = 0, s_leaf = 0;
    void *host_prob = nullptr, *host_split = nullptr;
    const void *tune_table = nullptr;
    uint64_t tune_version = 0;
    uint64_t groups = 0;
    bool operator==(const GraphKey &o) const {
        if (jobs_id != o.jobs_id || nd != o.nd || np != o.np || split != o.split || s_leaf != o.s_leaf ||
            host_prob != o.host_prob || host_split != o.host_split || tune_table != o.tune_table ||
            tune_version != o.tune_version || groups != o.groups)
            return false;
        for (int b = 0; b < B_COUNT; ++b)
            if (bufs[b] != o.bufs[b]) return false;
        return true;
    }
};

// One independent set of device buffers, stream and events on which the GPU pipeline runs.
// A context owns one; the serving loop gives every batch in flight its own.
struct Dev {
    hperm_opts opts{};                 // options of the current run (seed, plain chunk)
    hipStream_t stream = nullptr;
    DevBuf buf[B_COUNT];
    void *arena = nullptr;             // when set, every buffer is a slice of [arena, +arena_bytes)
    size_t arena_bytes = 0;
    size_t arena_required = 0;
    uint64_t resident_jobs = 0;        // id of the job table currently in B_DESC/B_DATA
    uint64_t resident_list = 0;        // id of the job table whose estimator list is in B_LIST
    void *resident_list_ptr = nullptr; // ... and where it was uploaded
    std::string last_error;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hperm_launch_stat> launches;   // R-NW launches of the last run
    std::vector<hipEvent_t> launch_ev;         // event pairs for the launches (grown on demand)
    // state between run_enqueue and run_finish
    bool want_per_job = false;
    bool persistent = true;
    bool timed = false;                        // per-job work cycles recorded (B_CYCLES)
    int split_launch = -1;                     // index of the device H_per launch, or -1
    unsigned long long *host_split = nullptr;  // pinned: its counters (B_SPLIT)
    bool graphed = false;                      // the last run replayed a graph
    hipGraphExec_t graph_exec = nullptr;       // the captured device part of a persistent run
    GraphKey graph_key;
    uint64_t graph_captures = 0;
    std::vector<JobAcc> host_acc;              // per-job accumulators (per-job results only)
    ProbAcc *host_prob = nullptr;              // pinned, per-problem accumulators
    size_t host_prob_cap = 0;
    std::vector<uint32_t> h_queue;             // host sources of the run's uploads
    std::vector<uint64_t> h_items;
    std::vector<JobDesc> h_desc_plain;
    std::shared_ptr<TuneTable> tune;           // tuned launch settings (shared by the context's pipelines)
};

// Release the buffers (owned ones freed), the events and the pinned staging memory.
void dev_release(Dev *d);

}  // namespace hp

struct hperm_ctx {
    hperm_opts opts;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool host_only = false;   // created by hperm_ctx_create_host: no device, no stream
    int device = 0;
    int num_cus = 0;
    hp::Dev dev;              // the context's own pipeline buffers
    hp::Serving *serving = nullptr;   // owned; created by hperm_serve_start
    std::mutex call_mu;       // serialises GPU pipelines of this context
};

namespace hp {

// Pipeline steps shared by the blocking calls and the serving loop (api.cpp).
hperm_status ensure_buf(Dev *c, BufId id, size_t bytes);
hperm_status upload_jobs(Dev *c, hperm_jobs *j);
hperm_status estimate_jobs(Dev *c, hperm_jobs *j, int trials, uint64_t seed);
// Launch steps 4-6 of all jobs on c->stream without waiting (results staged in c).
hperm_status run_enqueue(Dev *c, hperm_jobs *j, int order, int persistent, bool want_per_job);
// Bound on the leaves above order 16 that the device continuation of H_per may defer for
// these jobs under these options (0 when it is off).
uint64_t split_wide_total(const std::vector<JobDesc> &desc, const hperm_opts &o);
// Wait for c->stream and turn the staged accumulators into results.
hperm_status run_finish(Dev *c, hperm_jobs *j, hperm_result *per_job, hperm_result *totals,
                        double *t_rnw);
hperm_status run_jobs(Dev *c, hperm_jobs *j, int order, int persistent, hperm_result *per_job,
                      hperm_result *totals, double *t_rnw);
// Counters of one device expansion (dexpand_host.cpp).
struct DexpStats {
    uint64_t jobs = 0;             // nodes of the job order handed to the device H_per
    uint64_t nodes = 0;            // nodes written by the expansion (all levels)
    uint64_t max_level_nodes = 0;  // the most nodes a level held at once
    uint64_t launches = 0, relaunches = 0;
    uint64_t leaves = 0, leaf_terms = 0, splits = 0, split_stops = 0, deferred = 0, deferred_bound = 0;
    double split_s = 0.0, total_s = 0.0;
};
// per(A) of one problem (n > T) with the whole expansion tree on the device: the expansion
// down to order T, then the device continuation of H_per to order t (7 <= t < T <= 24); the
// level buffers take about budget_bytes. Requires a proven bound below 2^102.
// With a sample, the first max_jobs jobs of the tree (in tree order, the depth-first order of
// the expansion) are kept as dense T x T matrices with their exact values; stop_early ends the
// run once they are in (complete then reports whether the whole tree was evaluated).
struct DexpSample {
    uint64_t max_jobs = 0;
    bool stop_early = false;
    bool complete = false;
    std::vector<uint32_t> mats;
    std::vector<U512> vals;
};
hperm_status device_expand_problem(Dev *c, const CsrView &a, int T, int t, int s_leaf, size_t budget_bytes, U512 *out,
                                   DexpStats *stats, DexpSample *sample = nullptr);
// The same for several problems of one order n > T at once: their trees share the level
// buffers and the launches; out[k] receives per(A_k). moduli (one prime below 2^18 per problem,
// with n (p - 1) < 2^24): modular mode, out[k] = per(A_k) mod moduli[k] (entries reduced on
// entry; no bound applies); problems under different primes share the pass.
hperm_status device_expand_group(Dev *c, const std::vector<CsrView> &probs, int T, int t, int s_leaf,
                                 size_t budget_bytes, std::vector<U512> *out, DexpStats *stats,
                                 DexpSample *sample = nullptr, const std::vector<uint32_t> *moduli = nullptr);
// The largest modulus of modular mode for order n: min(2^18, (2^24 - 1) / n + 1).
uint32_t residue_prime_limit(int n);
// log2 of min(prod of row sums, prod of column sums), a bound on per(A) (0 for a zero line).
double residue_bound_bits(const CsrView &a);
// per(A_k) exactly for problems of one order n > T without the exact path's limits (entries and
// bound): the device path in modular mode modulo K + 1 primes below residue_prime_limit(n), K of
// them covering min(prod row sums, prod column sums), rebuilt by the Chinese remainder theorem
// and checked against the last, in one device pass (each problem once per prime). *nprimes
// receives K + 1.
hperm_status device_expand_residues(Dev *c, const std::vector<CsrView> &probs, int T, int t, int s_leaf,
                                    size_t budget_bytes, std::vector<U512> *out, DexpStats *stats, int *nprimes);

// The split order and the device expansion's job order in effect (0: off), and whether a
// problem takes the device expansion (api.cpp).
int split_in_effect(const hperm_opts &o);
int device_in_effect(const hperm_opts &o);
bool device_path(const hperm_opts &o, const CsrView &v);
// Whether the residue evaluation takes a problem of order n the exact paths refuse for range.
bool residue_path(const hperm_opts &o, int n);

// per(A) of a problem from its device accumulator (limb sums + CRT of the residue sums).
U512 prob_value(const ProbAcc &q);
void fill_result(const U512 &v, hperm_result *r);
// Work items of a job of order m with lane chunk 2^c (64 lanes per item).
uint64_t job_items(int m, int c);
// Device address of this device's no-allocation scratch array, looked up once per device
// (noalloc.hip); nullptr when the lookup failed.
void *noalloc_scratch(int device);
hperm_status set_error(Dev *c, hperm_status s, const std::string &msg);
hperm_status set_error(hperm_ctx *c, hperm_status s, const std::string &msg);
hperm_status hip_check(Dev *c, hipError_t e, const char *what);
ExpandParams expand_params(const hperm_opts &o);
void serve_shutdown(hperm_ctx *c);   // serve.cpp: stop the serving loop if running
uint64_t next_jobs_id();
double now_s();

}  // namespace hp
