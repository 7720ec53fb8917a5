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

// Device continuation of H_per (split.hip): jobs of order HP_SPLIT_MIN_T + 1 .. HP_SPLIT_MAX_M
// are split on the device down to order t (HP_SPLIT_MIN_T <= t < HP_SPLIT_MAX_M) and their
// leaves evaluated; each job's exact permanent per(B) lands in its accumulator as 32-bit limb
// sums flagged HP_ACC_NORMALISED (whatever its ring). The job's proven bound must stay below
// 2^102 (the leaves the 64-bit walk cannot take exactly are replayed modulo 2^128).
// stats[0..8) (cleared by the caller) receive leaves, leaf subset-terms, splits, splits refused
// by the entry bounds, deferred leaves, deferred leaves that found the record buffer full,
// leaves that failed their integrity check, and leaves deferred for want of a 64-bit bound; the
// last three must be 0 (else the result is not to be used). wide is a record buffer of
// split_wide_bytes(entries) bytes; two launches on stream s.
constexpr int HP_SPLIT_MAX_M = 24;
constexpr int HP_SPLIT_MIN_T = 7;
constexpr int HP_SPLIT_STATS = 8;
// Most leaves above order 16 a job of order m can defer: the nodes of orders 17..m.
inline uint64_t split_wide_entries(int m) { return m > 16 ? (1ull << (m - 16)) - 1 : 0; }
// Record buffer entries for jobs whose wide-leaf bounds sum to `wide`: room besides for one
// leaf per job deferred for want of a 64-bit bound (a job whose own bound admits it can defer
// at most its own root that way, when the rounding of the bound to float costs the margin).
inline uint64_t split_wide_capacity(uint64_t wide, uint64_t njobs) { return wide + njobs + 1024; }
size_t split_lds_bytes(int t, int mm);
// Resident waves (one per block) of the device H_per kernel for target t and job order mm.
int split_grid(int t, int mm);
size_t split_wide_bytes(uint64_t entries);
// Jobs of a host job table: queue[0..n) lists them (indices < njobs), mm is their largest order
// (> t), job_bound[job] their proven log2 bounds (float, rounded up); per-job values into accs;
// cycles (nullable) receives each job's shader-clock cycles.
hipError_t launch_split_jobs(const JobDesc *jobs, const uint32_t *data, const float *job_bound, const uint32_t *queue,
                             uint32_t n, uint32_t njobs, int t, int mm, int s_leaf, unsigned long long *head,
                             JobAcc *accs, unsigned long long *stats, void *wide, uint64_t wide_entries,
                             unsigned long long *cycles, hipStream_t s);
// Nodes of the device expansion: node k at nodes + node_off[k], k < n, all of order mm (> t);
// their values are summed into probs[problem of the node]; accs (nullable) receives each
// node's value.
// modp: 0 exact; else a prime below 2^18 and the nodes' values are taken modulo it (the nodes
// must come from a device expansion in the same modular mode).
hipError_t launch_split_nodes(const uint32_t *nodes, const uint64_t *node_off, uint32_t n, int t, int mm, int s_leaf,
                              unsigned long long *head, JobAcc *accs, ProbAcc *probs, unsigned long long *stats,
                              void *wide, uint64_t wide_entries, const uint32_t *modps, hipStream_t s);

}  // namespace hp
