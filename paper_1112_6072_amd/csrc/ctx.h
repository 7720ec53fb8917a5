// Context and job-table objects behind the C ABI of libhperm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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

enum BufId { B_DESC, B_DESC_PLAIN, B_DATA, B_KEYS, B_LIST, B_QUEUE, B_ITEMS, B_ACCS, B_HEAD, B_PROB, B_COUNT };

struct Serving;   // serve.cpp

}  // namespace hp

struct hperm_jobs {
    hp::JobTable tab;
    std::vector<float> keys;   // KKLLL keys, natural index
    bool has_keys = false;
    uint64_t id = 0;           // identity for device residency
};

struct hperm_ctx {
    hperm_opts opts;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool host_only = false;   // created by hperm_ctx_create_host: no device, no stream
    int device = 0;
    int num_cus = 0;
    hp::DevBuf buf[hp::B_COUNT];
    void *arena = nullptr;
    size_t arena_bytes = 0;
    size_t arena_required = 0;
    uint64_t resident_jobs = 0;   // id of the job table currently in B_DESC/B_DATA
    std::string last_error;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hp::Serving *serving = nullptr;   // owned; created by hperm_serve_start
    std::vector<hperm_launch_stat> launches;   // R-NW launches of the last call
    std::vector<hipEvent_t> launch_ev;         // event pairs for the launches (grown on demand)
    std::mutex call_mu;   // serialises GPU pipelines of this context (serving thread vs callers)
};

namespace hp {

// Pipeline steps shared by the blocking calls and the serving loop (api.cpp).
hperm_status ensure_buf(hperm_ctx *c, BufId id, size_t bytes);
hperm_status upload_jobs(hperm_ctx *c, hperm_jobs *j);
hperm_status estimate_jobs(hperm_ctx *c, hperm_jobs *j, int trials, uint64_t seed);
hperm_status run_jobs(hperm_ctx *c, hperm_jobs *j, int order, int persistent,
                      hperm_result *per_job, hperm_result *totals, double *t_rnw);
hperm_status set_error(hperm_ctx *c, hperm_status s, const std::string &msg);
hperm_status hip_check(hperm_ctx *c, hipError_t e, const char *what);
ExpandParams expand_params(const hperm_opts &o);
void serve_shutdown(hperm_ctx *c);   // serve.cpp: stop the serving loop if running
uint64_t next_jobs_id();
double now_s();

}  // namespace hp
