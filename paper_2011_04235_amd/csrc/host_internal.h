// Host-side structures shared by the reordering, the planner and the C ABI.
#pragma once

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fastpi.h"

namespace fastpi {

void set_error(const std::string& msg);

struct BlockDesc {
    int64_t row0, col0, rows, cols;
};

struct ReorderOut {
    std::vector<int32_t> piT, piF;
    std::vector<BlockDesc> blocks;
    int64_t m1 = 0, n1 = 0, m2 = 0, n2 = 0, iterations = 0, nnz_edges = 0;
};

// Validates the CSR pattern (and values when given). Returns FASTPI_OK or an error code
// with the message set.
int validate_csr(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col,
                 const double* val);

// Algorithm 2 (hub-and-spoke reordering) on the pattern; stored zeros are skipped when
// val is not null.
int reorder_pattern(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col,
                    const double* val, double k, ReorderOut& out);

int64_t target_rank(double alpha, int64_t x);

// One dense diagonal block of A11 as the device sees it. Work items are listed in the
// order the batched Jacobi launch takes them (largest cost first); the offsets address
// the packed outputs, which follow block order.
struct BlockWork {
    int64_t data_off;   // dense block, column-major rows x cols, in the block buffer
    int64_t u_off;      // U_i, column-major rows x s_i
    int64_t v_off;      // V_i, column-major cols x s_i
    int32_t rows, cols, rank, sig_off;   // sig_off: first column of the block in sigma1
    int32_t row0, col0, pad0, pad1;
};

// Work split of a compressed sparse structure (CSR or CSC, pointer array over `owners`
// rows or columns): every owner's entries are cut into segments of at most kSegLen entries.
// An owner with one segment is written directly; the segments of an owner with several
// write partial rows (pidx >= 0) that a second pass sums in segment order.
constexpr int64_t kSegLen = 64;
struct Segments {
    std::vector<int32_t> owner, pidx;
    std::vector<int64_t> begin, end;
    std::vector<int32_t> multi_owner;   // owners with several segments
    std::vector<int32_t> multi_ptr;     // their partial-row ranges (size multi_owner + 1)
    int64_t npart = 0;
};
void build_segments(const std::vector<int64_t>& ptr, Segments& out);

struct Plan {
    int64_t m = 0, n = 0, nnz = 0;   // nnz of the caller's CSR (including stored zeros)
    double alpha = 0, k = 0;
    ReorderOut ro;
    std::vector<int64_t> block_rank;     // s_i per block (all blocks)
    int64_t B_dense = 0, s_b = 0, s = 0, r = 0;
    std::vector<BlockWork> work;         // dense blocks, largest cost first
    int64_t blk_elems = 0, u1_elems = 0, v1_elems = 0;
    // Value maps: for caller nonzero e, dst0[e] and dst1[e] index the value buffer
    // [ dense blocks | A21 CSR | A21 CSC | T CSR | T CSC ], -1 = not written.
    std::vector<int64_t> dst0, dst1;
    int64_t off_a21r = 0, off_a21c = 0, off_tr = 0, off_tc = 0, val_elems = 0;
    // A21 (m2 x n1) and T (m x n2) patterns in new ids
    std::vector<int64_t> a21_rowptr, a21_colptr, t_rowptr, t_colptr;
    std::vector<int32_t> a21_colidx, a21_rowidx, t_colidx, t_rowidx;
    Segments seg_a21c, seg_a21r, seg_tc, seg_tr;   // A21 CSC/CSR, T CSC/CSR
    std::vector<int32_t> invT;   // new row -> original row
    std::vector<int32_t> invF;   // new column -> original column
};

// `given`: a reordering computed elsewhere (the GPU's) for this pattern and k, used instead
// of running the host one
int build_plan(Plan& p, int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col,
               const double* val, double alpha, double k, const ReorderOut* given = nullptr);
void assign_ranks(Plan& p, const std::vector<int64_t>& ranks);
int block_features(const Plan& p, const double* val, double* out);

// learned rank allocation (host arithmetic)
constexpr int kRankFeatures = 16;
void rank_inputs(int64_t n, const double* feats, const fastpi_rank_model& m, float* X, int32_t* ok);
void rank_allocate(int64_t n, const float* f, const int64_t* q, int64_t budget, int64_t* s);

}  // namespace fastpi
