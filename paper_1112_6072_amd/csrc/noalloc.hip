// The no-allocation entry point: per(A) of one small dense matrix evaluated as a single R-NW
// job, with every device buffer of the run (job descriptor and data, queue, queue heads, job
// and problem accumulators) carved from one file-scope device array instead of allocated.
//
// The array is looked up once per device with hipGetSymbolAddress (at context creation, with
// that device current) and only that address is handed to kernels and copies: in host code
// the array's name is a host-side stand-in, not a device address.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "ctx.h"
#include "kernels.h"

namespace hp {
namespace {

// Layout of the scratch array (byte offsets; 256-byte aligned regions).
constexpr size_t kOffDesc = 0;                          // one JobDesc
constexpr size_t kOffQueue = 256;                       // one job id
constexpr size_t kOffItems = 512;                       // one inclusive item count (u64)
constexpr size_t kOffHead = 768;                        // 8 queue heads (u64), cleared per call
constexpr size_t kOffAcc = kOffHead + 8 * 8;            // one JobAcc (64 B), cleared per call
constexpr size_t kOffProb = kOffAcc + sizeof(JobAcc);   // one ProbAcc (128 B), cleared per call
constexpr size_t kClearWords = (kOffProb + sizeof(ProbAcc) - kOffHead) / 8;
constexpr size_t kOffData = 1024;                       // the job's data block + 64 zero words
constexpr size_t kDataWordsMax = 5 * HP_MAX_M + HP_MAX_M * HP_MAX_M + HP_DATA_ALIGN + 64;
constexpr size_t kScratchBytes = 16384;
static_assert(kOffProb + sizeof(ProbAcc) <= kOffData, "scratch layout");
static_assert(kOffData + kDataWordsMax * 4 <= kScratchBytes, "scratch holds the largest job");

constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];
static bool g_scratch_done[kMaxDevices];

void *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        // called with `device` current (context creation)
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
        g_scratch_done[device] = true;
    }
    return g_scratch_ptr[device];
}

}  // namespace hp

using namespace hp;

extern "C" hperm_status hperm_permanent_dense_noalloc(hperm_ctx *c, int32_t n, const uint32_t *a,
                                                      hperm_result *out) {
    if (c && c->host_only) return set_error(c, HPERM_E_DEVICE, "host-only context");
    if (!c || !out) return HPERM_E_INVALID;
    if (c->serving) return set_error(c, HPERM_E_INVALID, "the context is serving");
    if (n < 0 || n > HP_MAX_M)
        return set_error(c, HPERM_E_INVALID, "the no-allocation call takes orders 0..40 (one job)");
    if (n > 0 && !a) return set_error(c, HPERM_E_INVALID, "a is null");
    std::lock_guard<std::mutex> lk(c->call_mu);
    const double t0 = now_s();
    hperm_result r;   // copied to *out only on success
    memset(&r, 0, sizeof(r));
    if (n == 0) {     // the empty product
        r.limb[0] = 1;
        r.nlimb = 1;
        r.t_total_s = now_s() - t0;
        *out = r;
        return HPERM_OK;
    }
    unsigned char *base = (unsigned char *)noalloc_scratch(c->device);
    if (!base) return set_error(c, HPERM_E_DEVICE, "hipGetSymbolAddress of the scratch array failed");

    JobDesc desc;
    uint32_t data[kDataWordsMax];
    size_t nwords = 0;
    double lb = 0.0;
    const int rc = pack_dense_job(n, a, c->opts.arith, &desc, data, kDataWordsMax - 64, &nwords, &lb);
    if (rc == -1) return set_error(c, HPERM_E_INVALID, "entries must be below 2^22");
    if (rc == -2) return set_error(c, HPERM_E_RANGE, "a row sum, the bound or the forced ring is out of range");
    if (rc == 1) {   // a zero row or column
        r.t_total_s = now_s() - t0;
        *out = r;
        return HPERM_OK;
    }
    for (size_t k = nwords; k < nwords + 64; ++k) data[k] = 0;   // lanes may read past a block
    const int m = desc.m;
    const int c_log2 = desc.chunk_log2;
    const int variant = walk_variant(desc, c_log2);
    const uint32_t job = 0;
    const uint64_t items = job_items(m, c_log2);
    hipStream_t s = c->stream;
    JobDesc *d_desc = (JobDesc *)(base + kOffDesc);
    uint32_t *d_queue = (uint32_t *)(base + kOffQueue);
    uint64_t *d_items = (uint64_t *)(base + kOffItems);
    unsigned long long *d_head = (unsigned long long *)(base + kOffHead);
    JobAcc *d_acc = (JobAcc *)(base + kOffAcc);
    ProbAcc *d_prob = (ProbAcc *)(base + kOffProb);
    uint32_t *d_data = (uint32_t *)(base + kOffData);
    hperm_status st;
    // inputs staged into the array (pageable sources: the copies finish before the calls
    // return their staging, and the stream is synchronised below before the stack unwinds)
    if ((st = hip_check(&c->dev, hipMemcpyAsync(d_desc, &desc, sizeof(desc), hipMemcpyHostToDevice, s), "stage job")))
        return st;
    if ((st = hip_check(&c->dev, hipMemcpyAsync(d_queue, &job, sizeof(job), hipMemcpyHostToDevice, s), "stage queue")))
        return st;
    if ((st = hip_check(&c->dev, hipMemcpyAsync(d_items, &items, sizeof(items), hipMemcpyHostToDevice, s),
                        "stage items")))
        return st;
    if ((st = hip_check(&c->dev, hipMemcpyAsync(d_data, data, (nwords + 64) * 4, hipMemcpyHostToDevice, s),
                        "stage job data")))
        return st;
    // every call starts from zeroed heads and accumulators (the array keeps the last call's)
    if ((st = hip_check(&c->dev, launch_fill_u64(d_head, kClearWords, 0ull, s), "clear scratch"))) return st;
    if ((st = hip_check(&c->dev,
                        launch_rnw_persistent(desc.arith, bucket_of(m), variant, d_desc, d_data, d_queue,
                                              (const uint64_t *)d_items, 1, items, d_head, d_acc, nullptr, 0, s),
                        "rnw_persistent launch")))
        return st;
    if ((st = hip_check(&c->dev, launch_recombine(d_desc, d_acc, 1, d_prob, s), "recombine launch"))) return st;
    ProbAcc q;
    if ((st = hip_check(&c->dev, hipMemcpyAsync(&q, d_prob, sizeof(q), hipMemcpyDeviceToHost, s), "download result")))
        return st;
    if ((st = hip_check(&c->dev, hipStreamSynchronize(s), "no-allocation run"))) return st;
    if (q.err) return set_error(c, HPERM_E_INTERNAL, "the job value failed its integrity check");
    const U512 v = prob_value(q);
    if (v.bits() > (int)std::ceil(lb) + 1) return set_error(c, HPERM_E_INTERNAL, "the result exceeds its proven bound");
    fill_result(v, &r);
    r.n_jobs = 1;
    r.max_m = m;
    r.arith_mask = 1 << (desc.arith + 1);
    r.subset_terms = 1ull << (m - 1);
    r.t_rnw_s = 0.0;
    r.t_total_s = now_s() - t0;
    *out = r;
    return HPERM_OK;
}
