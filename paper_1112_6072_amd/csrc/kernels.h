// Launchers of the HIP kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hperm_internal.h"

namespace hp {

// Order bucket of a job: the R-NW kernels are instantiated for m <= 16, 20, 24, 32, 40
// (HP_RNW_BUCKETS of them).
constexpr int HP_RNW_BUCKETS = 5;
int bucket_of(int m);

// Order bucket of the estimator: m <= 16, 20, 24, 32, 40 (HP_EST_BUCKETS of them).
constexpr int HP_EST_BUCKETS = 5;
int est_bucket_of(int m);

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, hipStream_t s);

// Normalise every job's accumulator and add it into its problem's accumulator.
hipError_t launch_recombine(const JobDesc *jobs, const JobAcc *accs, uint32_t njobs,
                            ProbAcc *probs, hipStream_t s);

// KKLLL keys of the listed jobs of one estimator bucket (one block of 4 waves per job);
// keys[job id].
hipError_t launch_estimate(int bucket, const JobDesc *jobs, const uint32_t *data,
                           const uint32_t *list, uint32_t nlist, int trials, uint64_t seed,
                           float *keys, hipStream_t s);

// Walk variant of a job for the R-NW kernels: 1 (2) for jobs whose Gray column 0 reaches at
// most the first 2 (exactly the first 3) rows and whose lane chunk holds at least 2 Gray
// indices (the paired walk), else 0.
int walk_variant(const JobDesc &d, int chunk_log2);

// Persistent R-NW over the queued jobs of one ring, order bucket and walk variant (queue[nqueue]
// job ids in scheduling order, item_end[nqueue] inclusive prefix sums of their item counts).
// *head must be 0. cycles (may be null): per-job work cycles are added into cycles[job id].
hipError_t launch_rnw_persistent(int ring, int bucket, int variant, const JobDesc *jobs,
                                 const uint32_t *data, const uint32_t *queue,
                                 const uint64_t *item_end, uint32_t nqueue, uint64_t total_items,
                                 unsigned long long *head, JobAcc *accs,
                                 unsigned long long *cycles, int grid_override, hipStream_t s);

// R-NW of one job in one launch (nitems waves).
hipError_t launch_rnw_single(int ring, int bucket, int variant, const JobDesc *jobs,
                             const uint32_t *data, uint32_t job, uint64_t nitems, JobAcc *accs,
                             hipStream_t s);

// Per-ring entry points (one object file per ring).
#define HP_RING_DECL(sfx)                                                                       \
    hipError_t persistent_grid_##sfx(int bucket, int variant, int *grid);                       \
    hipError_t launch_rnw_persistent_##sfx(int bucket, int variant, const JobDesc *jobs,        \
                                           const uint32_t *data, const uint32_t *queue,         \
                                           const uint64_t *item_end, uint32_t nqueue,           \
                                           uint64_t total_items, unsigned long long *head,      \
                                           JobAcc *accs, unsigned long long *cycles, int grid,  \
                                           hipStream_t s);                                      \
    hipError_t launch_rnw_single_##sfx(int bucket, int variant, const JobDesc *jobs,            \
                                       const uint32_t *data, uint32_t job, uint64_t nitems,     \
                                       JobAcc *accs, hipStream_t s);
HP_RING_DECL(w64)
HP_RING_DECL(w128)
HP_RING_DECL(res)
#undef HP_RING_DECL

// Resident grid (blocks) of the persistent kernel variant.
hipError_t persistent_grid(int ring, int bucket, int variant, int *grid);

// Device continuation of H_per (split.hip): mod-2^64 jobs of order HP_SPLIT_MIN_T + 1 ..
// HP_SPLIT_MAX_M are split on the device down to order t (HP_SPLIT_MIN_T <= t < HP_SPLIT_MAX_M)
// and their leaves evaluated; each job's value lands in accs[job].l[0] as for the R-NW
// kernels. queue[0..n) lists the jobs (indices < njobs), mm is their largest order (> t);
// head is a cleared counter; stats[0..6) (cleared by the caller) receive leaves, leaf
// subset-terms, splits, splits refused by the entry bounds, the wide leaves deferred to the
// second kernel, and deferred leaves that found the record buffer full (0 when the buffer holds
// split_wide_entries summed over the jobs); wide is a buffer of split_wide_bytes(entries)
// bytes; cycles (nullable) receives each job's shader-clock cycles (first kernel only). Two
// launches on stream s.
constexpr int HP_SPLIT_MAX_M = 24;
constexpr int HP_SPLIT_MIN_T = 7;
// Most leaves above order 16 a job of order m can defer: the nodes of orders 17..m.
inline uint64_t split_wide_entries(int m) { return m > 16 ? (1ull << (m - 16)) - 1 : 0; }
size_t split_lds_bytes(int t, int mm);
size_t split_wide_bytes(uint64_t entries);
hipError_t launch_split_w64(const JobDesc *jobs, const uint32_t *data, const uint32_t *queue, uint32_t n,
                            uint32_t njobs, int t, int mm, int s_leaf, unsigned long long *head, JobAcc *accs,
                            unsigned long long *stats, void *wide, uint64_t wide_entries,
                            unsigned long long *cycles, hipStream_t s);

}  // namespace hp
