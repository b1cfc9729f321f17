// Host-callable launchers of the HIP kernels (all stream-ordered, none synchronises unless
// stated).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "host_internal.h"

namespace fastpi {

// device view of a Segments table (pointers into device memory)
struct SegDev {
    const int32_t* owner;
    const int64_t* begin;
    const int64_t* end;
    const int32_t* pidx;
    const int32_t* multi_owner;
    const int32_t* multi_ptr;
    int64_t nseg, nmulti, npart;
};

// Per-launch timing of one kernel kind (measurement only). A timed launch goes through
// hipExtLaunchKernel with an event pair that the runtime stamps at the dispatch's own start
// and end, so the pair measures the kernel body (events recorded around a launch would also
// count its dispatch gap).
enum KernelKind {
    KT_NONE = -1,
    KT_EIG_GRAM = 0,
    KT_EIG_SOLVE = 1,
    KT_EIG_UPDATE = 2,
    KT_BLOCK_SVD = 3,
    KT_LABEL_SPMM = 4,
    KT_TOPK = 5,
    KT_GEMM_NT = 6,
    KT_SUB_GEMM = 7,   // products by G of the subspace core solver
    KT_CQ_PANEL = 8,   // panel kernel of the subspace solver's Cholesky QR
    KT_EIG_ROUND = 9,  // eigensolver column update and next round's partial Grams, one launch
    KT_LAST = KT_EIG_ROUND
};
struct KernelTimer {
    int target = KT_NONE;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    bool failed = false;
    hipEvent_t take() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                failed = true;
                return nullptr;
            }
            pool.push_back(e);
        }
        return pool[used++];
    }
    // an event pair for the next launch if `kind` is the timed one
    bool pair(int kind, hipEvent_t& e0, hipEvent_t& e1) {
        if (kind != target || failed) return false;
        e0 = take();
        e1 = e0 ? take() : nullptr;
        if (!e0 || !e1) {
            failed = true;
            return false;
        }
        return true;
    }
};

// launches `kernel`, timed when `timer` is set and times `kind`
#define FASTPI_LAUNCH(timer, kind, kernel, grid, block, shmem, st, ...)                               \
    do {                                                                                            \
        hipEvent_t fastpi_e0_, fastpi_e1_;                                                          \
        if ((timer) && (timer)->pair((kind), fastpi_e0_, fastpi_e1_))                               \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, fastpi_e0_, fastpi_e1_, 0u, __VA_ARGS__); \
        else                                                                                        \
            hipLaunchKernelGGL(kernel, grid, block, shmem, st, __VA_ARGS__);                        \
    } while (0)

// C = op(A) op(B) on the matrix cores (mfma_gemm.hip): op(A) = A (M x K) or, with ta, A stored
// K x M; op(B) = B (K x N) or, with tb, B stored N x K; FP64, or FP32 operands and
// accumulation with fp32; nsplit > 1 writes partial products of K chunks at C + z cstride.
void launch_mfma_gemm(bool ta, bool tb, const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M,
                      int64_t N, int64_t K, double* C, int64_t ldc, int nsplit, int64_t cstride, hipStream_t st,
                      bool fp32, KernelTimer* timer = nullptr, int kind = KT_NONE);
// C[crow(i)] = A[arow(i)] B on the matrix cores (row gather of A, row scatter of C; a null
// map is the identity), one K chunk
void launch_mfma_gemm_rows(const double* A, int64_t lda, const int* arow, const double* B, int64_t ldb, int64_t M,
                           int64_t N, int64_t K, double* C, int64_t ldc, const int* crow, hipStream_t st, bool fp32);

// C[i * ldc + j] = sum_z part[z][i][j] (z < nsplit, fixed order)
void launch_sum_parts(const double* part, int nsplit, int64_t M, int64_t N, double* C, int64_t ldc, hipStream_t st);

void launch_fill(double* p, int64_t n, double v, hipStream_t st);
void launch_fill_i32(int* p, int64_t n, int v, hipStream_t st);
void launch_gather(const double* val, const int64_t* dst0, const int64_t* dst1, int64_t nnz,
                   double* out, int* status, hipStream_t st);

// One diagonal block for the persistent block-SVD launch: absolute device addresses, so the
// blocks of several matrices can share one launch. `scratch` holds rows*cols + q*q elements
// of the compute type for blocks that do not fit the launch's LDS budget.
struct BlockTask {
    const double* A;    // dense block, column-major rows x cols
    double* U;          // rows x rank, column-major
    double* V;          // cols x rank, column-major
    double* sig;        // rank values, descending
    void* scratch;
    int* status;        // [0] status bits, [1] maximum sweeps used
    int32_t rows, cols, rank, pad;
};

// Persistent batched Jacobi: `grid` workgroups take tasks from an atomic queue (`counter`
// must hold 0 at launch; the launcher clears it with a fill kernel first).
void launch_block_svd_tasks(bool fp32, const BlockTask* tasks, int ntasks, int* counter,
                            int lds_bytes, int grid, int max_sweeps, double tol_scale,
                            hipStream_t st, KernelTimer* timer = nullptr);
void launch_copy(const double* src, int64_t n, double* dst, hipStream_t st);

// eigensolver (eig.hip): block one-sided Jacobi on a set of independent symmetric PSD
// problems ("jobs") that advance together, one launch per kernel and round for all jobs.
struct EigJob {
    const double* G;    // q x q row-major input
    double* A;          // q x q scratch of the pivoted Cholesky (may be G itself), or null
    double* vals;       // t eigenvalues, descending
    double* vecs;       // q x t row-major eigenvectors
    double* X;          // ld x ld column-major iterate
    double* Xs;         // ld x ld: the reordered columns, then the second iterate of the fused
                        // rounds; null above order 16384 (no reordering, three launches a round)
    double* Hpart;      // npairs * nchunk partial 32 x 32 Grams
    double* W;          // 2 * npairs 32 x 32 rotations (by round parity)
    double* lam;        // ld column norms, then the noise floor
    int* flag;          // 2 * npairs: pair rotated in this round (by round parity)
    int* order;         // t: columns of the t largest norms
    int* perm;          // ld: the columns of X by descending norm (column order of the next sweep)
    int* status;        // status word of the owner (bit 1 when the sweep cap is hit), or null
    double tol;         // cosine threshold of the outer pairs
    int64_t q, t, ld;
    int nblk, nbe, npairs, nchunk, nupd, tag;
    int squared;        // X = R^T of a pivoted Cholesky (the job's start; set by the set from
                        // the set's choice and the job's scratch A): eigenvalues are squared
                        // column norms
    int pad;
};
// Cholesky QR of the subspace core solver (subspace.hip): one job per core and call.
// B (kp x kp row-major, kp = k rounded up to 64) holds Y^T Y in [0, k)^2 and the identity
// beyond (zero off the diagonal, set once); its lower triangle is overwritten by L. M
// (kp x kp, zero above the diagonal, set once) receives L^-1; dg (kp) is B's diagonal before
// the factorisation; flag (device int) is or-ed with 1 when a pivot shows numerical rank
// loss.
struct CholJob {
    double* B;
    double* M;
    double* dg;
    int* flag;
    int k, kp;
};
void launch_chol_inverse(const CholJob* jobs, int njobs, int max_kp, hipStream_t st, KernelTimer* timer = nullptr);
// flag |= 1 when a column of R = G V (q x t) leaves lam_i V[:, i] by more than tol * lam_0
void launch_sub_residual(const double* R, const double* V, const double* lam, int64_t q, int64_t t, double tol,
                         int* flag, hipStream_t st);
void launch_symmetrize(double* H, int64_t k, hipStream_t st);
// p[i * ld + i] = v for i in [i0, i1)
void launch_fill_diag(double* p, int64_t ld, int64_t i0, int64_t i1, double v, hipStream_t st);

// per-job device state words of an EigSet (then one all-done word after the last job)
constexpr int kEigStRot = 0;      // pairs rotated in the current sweep
constexpr int kEigStDone = 1;     // converged or capped
constexpr int kEigStSweeps = 2;   // sweeps run
constexpr int kEigStCapped = 3;   // stopped by the sweep cap
constexpr int kEigStTotal = 4;    // pairs rotated over all finished sweeps
constexpr int kEigStateWords = 6;
struct EigSet {
    int njobs = 0, rounds = 0, gram_rows = 128;
    EigJob* jobs = nullptr;       // device, jobs sorted by rounds per sweep (descending)
    int* pre = nullptr;           // device prefix sums of the per-job workgroup counts:
                                  // gram, solve, update (each njobs + 1)
    int* state = nullptr;         // device, kEigStateWords per job, then the all-done word
    int* host_state = nullptr;    // pinned mirror of state
    int* pstate = nullptr;        // device, per job {pivots taken, factorisation done}
    int precond = 0;              // start from the pivoted Cholesky factor instead of G
    int fused = 0;                // two launches per round (every job has its second iterate Xs)
    std::vector<EigJob> host;     // host copy, same order
    std::vector<int> nact, g_gram, g_solve, g_upd;   // per round: active jobs and grids
    int64_t max_ld = 0, max_q = 0;
};
int64_t eig_padded_order(int64_t q);
int eig_gram_rows_valid(int rows);
size_t eig_job_doubles(int64_t q, int gram_rows);
size_t eig_job_ints(int64_t q);
// A: writable q x q scratch for the pivoted-Cholesky preconditioner (may alias G), or null
EigJob eig_make_job(const double* G, double* A, int64_t q, int64_t t, double* vals, double* vecs,
                    double* ws, int* iws, int* status, double tol, int gram_rows, int tag);
// precond: factor the G of every job that has scratch A first and iterate on its R^T (jobs
// without A start from G)
// fused: two launches per round where every job allows it (else three)
int eig_set_create(EigSet& es, std::vector<EigJob> jobs, int gram_rows, bool precond, bool fused,
                   hipStream_t st);
// pivoted Cholesky of every job of the set into its X (pchol.hip)
void pchol_run(const EigSet& es, hipStream_t st);
void eig_set_free(EigSet& es);
void eig_begin(const EigSet& es, hipStream_t st);
void eig_sweep(const EigSet& es, int max_sweeps, int inner_sweeps, hipStream_t st,
               KernelTimer* timer);
void eig_end(const EigSet& es, hipStream_t st);
// Runs sweeps (eagerly, or by replaying `sweep_graph`) until every job is done; the state of
// sweep k is read on copy_st while sweep k+1 is queued. On return es.host_state is final.
int eig_iterate(const EigSet& es, int max_sweeps, int inner_sweeps, hipStream_t st,
                hipStream_t copy_st, KernelTimer* timer, hipGraphExec_t sweep_graph);

// dense (dense.hip)
// K split of a transposed-A product (M x N over K) for launch_gemm_tn in the given precision
int gemm_tn_splits(int64_t M, int64_t N, int64_t K, bool fp32 = false, int ncu = 256);
void launch_gemm_tn(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M,
                    int64_t N, int64_t K, double* C, int64_t ldc, const double* rs,
                    const double* cs, double* part, int nsplit, hipStream_t st, bool fp32 = false);
void launch_gemm_nn(const double* A, int64_t lda, const int* arow, const double* B, int64_t ldb,
                    int64_t M, int64_t N, int64_t K, double* C, int64_t ldc, const int* crow,
                    hipStream_t st, bool fp32 = false, KernelTimer* timer = nullptr, int kind = KT_NONE);
void launch_gemm_nt(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N,
                    int64_t K, double* C, int64_t ldc, hipStream_t st, bool fp32 = false,
                    KernelTimer* timer = nullptr);

// sparse and block-structured (sparse.hip)
void launch_sparse_gram(const SegDev& sg, const int* rowidx, const double* cval,
                        const int64_t* rowptr, const int* colidx, const double* rval, int64_t q,
                        double* G, int64_t ldg, bool accumulate, double* part, hipStream_t st);
void launch_sparse_proj(const SegDev& sg, const int* rowidx, const double* cval, const double* U,
                        int64_t s, const double* sigma, double* G, int64_t ldg, int64_t off,
                        double* part, hipStream_t st);
// Label SpMM over row blocks of the labelled rows (at most kLabelBlockRows rows and
// kLabelBlockPos positives a block): C (L x r) = cs .* (Y^T U). Frequent labels are split into
// sub-labels (label l: vbase[l] .. vbase[l+1] - 1, Lv in all, at most label_slots(L)); each
// block lists its (sub-label, run) pairs; chunks of blocks are summed through part
// (label_spmm_chunks(nblk, r, Lv) x Lv x r).
constexpr int kLabelBlockRows = 256;
constexpr int kLabelBlockPos = 4096;
constexpr int kLabelSubGroup = 2048;   // sub-labels of one workgroup (accumulated in LDS)
struct LabelBlocks {
    const int32_t* lrows = nullptr;   // labelled rows, increasing (nl)
    const int32_t* bstart = nullptr;  // first labelled row of each block (nblk + 1)
    const int32_t* bbase = nullptr;   // first entry of each block in prow / pval, 16-aligned (nblk + 1)
    const int32_t* rg = nullptr;      // first run of each (block, sub-label group) (nblk * (groups + 1))
    const int32_t* rv = nullptr;      // sub-label of each run
    const int32_t* re = nullptr;      // first entry of each run, relative to bbase (a sentinel ends a block)
    const uint8_t* prow = nullptr;    // row within the block of each entry
    const double* pval = nullptr;     // values, or null when every value is 1
    const int32_t* vbase = nullptr;   // sub-labels of each label (L + 1)
    int64_t nblk = 0, Lv = 0;
};
int label_spmm_chunks(int64_t nblk, int64_t r, int64_t Lv);
int label_slots(int64_t L);
int label_groups(int64_t Lv);
void launch_label_spmm(const LabelBlocks& lb, const double* U, int64_t r, int64_t L, const double* cs, double* C,
                       double* part, hipStream_t st, KernelTimer* timer);
void launch_spmm_rows(const SegDev& sg, const int* colidx, const double* rval, const double* B,
                      int64_t N, const double* cs, double* C, int64_t ldc, const int* crow,
                      bool accumulate, double* part, hipStream_t st, KernelTimer* timer = nullptr);
void launch_blockdiag_gram(const BlockWork* work, int nwork, const double* V1, const double* sig1,
                           double* G, int64_t ldg, hipStream_t st);
void launch_u2_top(const BlockWork* work, int nwork, const double* U1, const double* sig1,
                   const double* V1, const double* V2, int64_t s, const double* inv_sig2,
                   double* U2, int* status, hipStream_t st);
// Status word bits of one matrix: 1 non-finite value, 2 sweep cap reached, 4 internal bound,
// 8 a kept singular value under the Gram floor (warning).
constexpr int kStatusFloor = 8;
void launch_sqrt_inv(const double* lam, int64_t t, double rel_cut, double* sigma, double* inv, int* status,
                     hipStream_t st);
void launch_col_coeffs(const double* Vt, int64_t s, int64_t n2, int64_t r, const double* sig2,
                       const double* inv3, double* C1, double* C2, hipStream_t st);
void launch_copy_rows(const double* src, int64_t rows, int64_t cols, const int* dst_row, double* dst,
                      hipStream_t st);
void launch_pinv_sigma(const double* S, int64_t r, double cut, double* inv, hipStream_t st);

// randomized inner solver (randomized.hip): out[0..count) standard normals from Philox4x32-10
// with key (seed, stream) (row-major; pair e/2 per counter, Box-Muller); S = V diag(d^-1/2)
// over the eigenpairs (d descending) with d_j > cut * d_0, zero columns elsewhere.
void launch_gauss(double* out, int64_t count, uint32_t seed, uint32_t stream, hipStream_t st);
void launch_scale_cols(const double* V, const double* d, int64_t k, double cut, double* S, hipStream_t st);
// Outputs of a block SVD computed through its Gram matrix: sigma_k = sqrt(lam_k) (0 when
// lam_k <= (cut sigma_0)^2, with kStatusFloor set in *status when sigma_0 > 0), the q-side
// factor E[:, k] (E: q x t row-major) and the p-side factor W[:, k] / sigma_k (W: p x t
// row-major; 0 for a zero sigma), both written column-major into the block's packed outputs.
void launch_block_gram_out(const double* lam, const double* E, const double* W, int64_t q, int64_t p,
                           int64_t t, double cut, double* qout, double* pout, double* sig, int* status,
                           hipStream_t st);
// negates each column of V (rows x cols, row-major) whose largest-magnitude entry (first on
// ties) is negative
void launch_sign_fix(double* V, int64_t rows, int64_t cols, hipStream_t st);

// GPU reordering (reorder_gpu.hip): Algorithm 2 on a device CSR with the host reordering's
// result (piT, piF, blocks, split); validate_csr_gpu checks a device CSR first (shape,
// column range and order, finite values).
int validate_csr_gpu(int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col,
                     const double* val, hipStream_t st);
int reorder_pattern_gpu(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                        int64_t nnz, double k, hipStream_t st, ReorderOut& out);

// label evaluation (evaluate.hip): for every row x of a sparse test matrix (CSR over n
// columns), scores s = x Z (Z: n x L row-major), the kmax highest labels (ties to the lower
// label) and hits[row * nk + t] = |top ks[t] labels ∩ the row's true labels (CSR)|; a row
// with a column outside [0, n) gets -1 counts. ks_host: host array of nk values in
// [1, kTopkMaxK]; kmax = max(ks). The scores of a chunk of rows go to `scratch`
// (topk_scratch_doubles(rows, L) doubles, at most kTopkScoreDoubles or one row).
constexpr int kTopkMaxK = 64;
constexpr int kTopkMaxKs = 16;
constexpr int64_t kTopkScoreDoubles = int64_t(32) << 20;
int64_t topk_scratch_doubles(int64_t rows, int64_t L);
void launch_topk_hits(int64_t rows, int64_t n, int64_t L, const int64_t* a_rowptr, const int* a_col,
                      const double* a_val, const double* Z, const int64_t* y_rowptr, const int* y_col,
                      int nk, const int* ks_host, int kmax, int* hits, double* scratch, hipStream_t st,
                      KernelTimer* timer = nullptr);

// rank predictor (mlp.hip)
int mlp_param_count();
size_t mlp_scratch_floats(int64_t N);
void launch_mlp_forward(int64_t N, const float* X, const float* th, float* f, float* act,
                        hipStream_t st);
void launch_mlp_gradient(int64_t N, const float* X, const float* y, const float* th, float* grad,
                         float* scratch, hipStream_t st);
void launch_mlp_adam(float* th, const float* g, float* m, float* v, int64_t step, float lr,
                     hipStream_t st);

}  // namespace fastpi
