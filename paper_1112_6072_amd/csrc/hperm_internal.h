// Internal layout shared by the host code and the HIP kernels of libhperm.
//
// A job is one sub-matrix B of order m (1..HP_MAX_M) produced by expansion (2) of the
// paper. R-NW evaluates it with Ryser's formula in Nijenhuis-Wilf form (Introduction):
// one column of B (the densest, index m-1 after reordering) is fixed, the other m-1
// "Gray columns" are enumerated by a binary-reflected Gray code. With doubled factors
//     f_i(S) = base_i + 2 * sum_{j in S} b_ij,   base_i = 2 b_{i,m-1} - R_i,
// (R_i the row sum of B) the kernels compute the ring value
//     V = sum_{k=0}^{2^(m-1)-1} (-1)^k prod_i f_i(gray(k)) = (-1)^(m-1) 2^(m-1) per(B).
#pragma once
#include <stdint.h>

#define HP_MAX_M 40          // largest job order the kernels accept
#define HP_MAX_N 128         // largest input order
#define HP_MAX_ENTRY (1u << 22)   // expanded entries stay below this (2*b is a 24-bit signed value)
#define HP_MAX_ROWSUM (1u << 24)  // row sums stay below this, so |f_i| < 2^24

// Arithmetic rings of the kernels (values of JobDesc::arith).
enum : uint8_t { HP_W64 = 0, HP_W128 = 1, HP_RES = 2, HP_NRING = 3 };

// Residue primes p_k = 2^61 - c_k (all three verified prime by the tests).
#define HP_P_BITS 61
#define HP_C0 1ull
#define HP_C1 31ull
#define HP_C2 45ull

// One job, 16 bytes, in the device job table.
//   data_off : offset (in 32-bit words) of the job's data block in the data array
//   m        : order; the job has m-1 Gray columns
//   arith    : HP_W64 / HP_W128 / HP_RES
//   chunk_log2 : Gray indices per lane in one work item = 2^chunk_log2
//   nnz      : number of entries in the Gray columns
//   problem  : input problem the job belongs to
// Rows are sorted by level (the first Gray column that touches them); a flip of Gray column
// j changes only rows below hi[j].
// Data block (32-bit words, starting at data_off):
//   [0, m)            base_i as int32
//   [m, 2m)           col_start[j] for j = 0..m-1: entry offset (relative to the entry
//                     block) of Gray column j; col_start[m-1] = nnz (end)
//   [2m, 3m)          hi[j]: 1 + the lowest job row of Gray column j (hi[m-1] = m)
//   [3m, 3m+nnz)      entries of Gray column 0, then 1, ...: (2*b_ij << 8) | i
//   [3m+nnz, 4m+nnz)  original column index of Gray column g (g < m-1) and of the fixed
//                     column (slot m-1)
//   [4m+nnz, 5m+nnz)  original row index of job row i
//                     (the last two are used only for the estimator's random draws)
struct JobDesc {
    uint32_t data_off;   // start of the job's data block in units of HP_DATA_ALIGN words
    uint8_t m;
    uint8_t arith;
    uint8_t chunk_log2;
    uint8_t flags;       // HP_FLAG_* bits
    uint32_t nnz;
    uint32_t problem;
};
static_assert(sizeof(JobDesc) == 16, "JobDesc layout");

// JobDesc::flags: Gray column 0 reaches only job rows 0 and 1 (hi[0] <= 2); the job holds
// the transpose of the expansion's sub-matrix (same permanent; the estimator then swaps row
// and column in its draws so that they follow the sub-matrix).
constexpr uint8_t HP_FLAG_COL0_TWO_ROWS = 1;
constexpr uint8_t HP_FLAG_COL0_THREE_ROWS = 2;   // hi[0] = 3
constexpr uint8_t HP_FLAG_TRANSPOSED = 4;
// mod 2^64 jobs of order >= 5 whose Gray column 0 touches rows 0..1 and column 1 only rows
// 2..hi[1]-1 with hi[1] = 4 or 5: the four-step walk applies
constexpr uint8_t HP_FLAG_QUAD = 8;

static inline uint32_t hp_job_words(int m, int nnz) { return 5u * (uint32_t)m + (uint32_t)nnz; }

// Data blocks start at multiples of 4 words (16 bytes), so that a 32-bit data_off reaches
// 2^34 words (64 GiB of job data).
constexpr uint32_t HP_DATA_ALIGN = 4;
static inline size_t hp_data_index(const JobDesc &d) { return (size_t)d.data_off * HP_DATA_ALIGN; }
static inline size_t hp_align_words(size_t n) { return (n + HP_DATA_ALIGN - 1) / HP_DATA_ALIGN * HP_DATA_ALIGN; }

// Per-job accumulator of the kernels: sums of 32-bit limbs of the work items' ring values
// (integer addition is associative, so the atomic order does not change the result):
//   W64  : l[0] = V mod 2^64 (wrap-around sum of the items' values)
//   W128 : V = sum_k l[k] 2^(32k) mod 2^128, k = 0..3 (limb k of each item, summed)
//   RES  : V mod p_k = (l[2k] + 2^32 l[2k+1]) mod p_k (low and high halves of residues)
//   normalised (flag == HP_ACC_NORMALISED, written by the device continuation of H_per):
//          per(B) itself = sum_k l[k] 2^(32k), k = 0..3, whatever the job's ring
struct JobAcc {
    unsigned long long l[6];
    unsigned long long flag;
    unsigned long long pad;
};
constexpr unsigned long long HP_ACC_NORMALISED = 1;
static_assert(sizeof(JobAcc) == 64, "JobAcc layout");

// A sub-matrix node of the device expansion (one per node, 16-byte aligned, 32-bit words):
//   w[0]  order o (bits 0..7) | nnz << 8
//   w[1]  proven upper bound of log2 per(node), as float bits (the smallest of the bounds of
//         the node's ancestors and its own row-sum bound; per(child) <= per(parent) since all
//         entries are non-negative)
//   w[2]  problem index
//   w[3]  zero
//   w[4 .. 4 + ceil(o/4))  row lengths, one byte per row (row i: byte i % 4 of word 4 + i / 4)
//   then the nnz entries row by row, columns increasing: (value << 8) | column
#if defined(__HIPCC__)
#define HP_HOST_DEVICE __host__ __device__
#else
#define HP_HOST_DEVICE
#endif
HP_HOST_DEVICE static inline uint32_t hp_node_words(int o, int nnz) {
    return (4u + ((uint32_t)o + 3u) / 4u + (uint32_t)nnz + 3u) & ~3u;
}

// Per-problem accumulator of the device recombination: lim[k] sums limb k (32 bits) of the
// exact permanents of the problem's 2-adic-ring jobs; res[2k], res[2k+1] sum the low and
// high 32-bit halves of the residues mod p_k of its residue-ring jobs; err is set when a
// job fails its 2-adic integrity check.
struct ProbAcc {
    unsigned long long lim[4];
    unsigned long long res[6];
    unsigned int err;
    unsigned int pad[11];
};
static_assert(sizeof(ProbAcc) == 128, "ProbAcc layout");
