// Host side of the path: validation, expansion (2) into jobs, bounds and job packing.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "hperm_internal.h"

namespace hp {

struct ExpandParams {
    int m_cut = 20;
    int m_cap = 36;
    int s_leaf = 5;
    int arith = 0;        // hperm_arith: 0 auto, 1 W64, 2 W128, 3 RES
    int chunk_log2 = 0;   // 0: table
    int threads = 0;
    size_t max_bytes = 0;   // host job-table limit (descriptors, data, bounds); 0: none
};

// Host copy of the job table of one or more problems.
struct JobTable {
    std::vector<JobDesc> desc;        // natural (expansion) order
    std::vector<uint32_t> data;       // data blocks
    std::vector<double> log2_bound;   // proven log2 upper bound of each job's permanent
    int n_problems = 0;
    // per problem: exact value known without GPU work (n = 0, tiny problems) and whether
    // the problem is identically zero
    std::vector<int> direct_valid;
    std::vector<uint64_t> direct_value;   // valid when direct_valid (value < 2^64)
    std::vector<double> problem_log2_bound;
};

struct CsrView {
    int n;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const uint32_t *val;
};

// Validate a CSR matrix (sizes, ordering). Empty string if fine, else the reason.
std::string validate_csr(const CsrView &a);

// Expand problems into jobs and append them to *out (out->n_problems grows by the count).
// Returns 0 on success, or -1 (invalid), -2 (range) or -3 (the job table would exceed
// prm.max_bytes) with *err set.
int expand_problems(const std::vector<CsrView> &probs, const ExpandParams &prm, JobTable *out,
                    std::string *err);

// Turn dense matrices directly into jobs (no expansion), one problem each.
int jobs_from_dense(int count, const int32_t *m, const int64_t *off, const uint32_t *a,
                    const ExpandParams &prm, JobTable *out, std::string *err);

// One dense matrix of order n (1..HP_MAX_M) packed as a single job without heap allocation
// (the packing of jobs_from_dense, problem 0): *desc, data[0..*nwords) (data_off 0; at most
// fixed_job_words() words), *log2b the proven bound. Returns 0, 1 (a zero line: per = 0, no
// job), -1 (invalid argument or entry >= 2^22) or -2 (range: row sum, bound, forced ring).
size_t fixed_job_words();
int pack_dense_job(int n, const uint32_t *a, int arith, JobDesc *desc, uint32_t *data, size_t cap_words,
                   size_t *nwords, double *log2b);

// The root node of the device expansion (hp_node_words layout, problem 0) of a validated CSR
// matrix, and its proven log2 bound. Returns 0, 1 (a zero row or column: per = 0) or -2 (an
// entry or row sum beyond the kernels' limits).
int pack_root_node(const CsrView &a, std::vector<uint32_t> *node, double *log2b);

// Knuth's random-descent estimate of the expansion tree of a validated CSR matrix under the
// rule of the device path (split every node above order T, then H_per's rule down to order
// t): nodes[o] and leaves[o] (o = 0..n) receive the estimated nodes and leaves of each order.
// Returns 0, or -2 when an expanded entry leaves the supported range on a sampled path.
int estimate_tree(const CsrView &a, int T, int t, int s_leaf, int samples, uint64_t seed, double *nodes,
                  double *leaves);

// Default lane chunk (log2 Gray indices per lane) for a job of order m.
int default_chunk_log2(int m);

}  // namespace hp
