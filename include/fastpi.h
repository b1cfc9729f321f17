/*
 * fastpi.h -- C ABI of the MI355X FastPI library (low-rank SVD of a reordered sparse
 * feature matrix and the pseudoinverse apply), after Jung & Sael, "Fast and Accurate
 * Pseudoinverse with Sparse Matrix Reordering and Incremental Approach" (arXiv 2011.04235).
 *
 * The library computes A ~= U Sigma V^T for a sparse A (m x n, CSR) and a rank ratio
 * alpha in (0, 1] (Algorithm 1, lines 1-4), and then Z = V Sigma^+ U^T Y for a label
 * matrix Y (Problem 1 with Application 1).
 *
 * Conventions for every call below:
 *  - indices are 0-based; dense matrices are row-major (C order) with the stated shape;
 *  - "host" pointers are ordinary CPU memory, "device" pointers are HIP device memory of
 *    the handle's device; the caller owns every buffer passed in and the library never
 *    frees or keeps caller memory beyond the call (except where a plan is uploaded);
 *  - device calls are ordered on the handle's HIP stream and return before the device has
 *    finished; fastpi_sync() waits and reports device-side failures;
 *  - each call returns a fastpi_status; after an error the outputs are unspecified and
 *    fastpi_last_error() returns a message for the calling thread;
 *  - a handle is bound to one stream and must not be used from two threads at once.
 */
#ifndef FASTPI_H
#define FASTPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FASTPI_WFLOOR = 1,       /* warning, outputs valid: a kept singular value lay at or below  */
                             /* the Gram route's resolution floor and is returned as 0 (see    */
                             /* fastpi_svd); reported by fastpi_sync / fastpi_batch_sync only  */
    FASTPI_OK = 0,
    FASTPI_EINVAL = -1,      /* bad argument: null pointer, alpha or k out of range, bad id   */
    FASTPI_ESHAPE = -2,      /* CSR not well formed: rowptr not monotone, column out of range, */
                             /* columns not strictly increasing within a row                  */
    FASTPI_ENONFINITE = -3,  /* a stored value is NaN or infinite                              */
    FASTPI_ENOMEM = -4,      /* device or host allocation failed, or the workspace cap is hit  */
    FASTPI_EHIP = -5,        /* a HIP runtime call failed                                      */
    FASTPI_ENOCONV = -6,     /* a Jacobi iteration reached its sweep cap before converging    */
    FASTPI_EINTERNAL = -7
} fastpi_status;

typedef enum { FASTPI_FP64 = 0, FASTPI_MIXED = 1 } fastpi_precision;

/* Shape report of a plan (symbols of Table 1). */
typedef struct {
    int64_t m, n;        /* rows (instances) and columns (features) of A                     */
    int64_t nnz;         /* stored non-zeros used as edges (explicit zeros are dropped)      */
    int64_t m1, n1;      /* spoke rows and columns: the size of A11                          */
    int64_t m2, n2;      /* hub rows and columns                                             */
    int64_t B;           /* diagonal blocks of A11, including blocks of height or width 0    */
    int64_t B_dense;     /* blocks with both height and width > 0                            */
    int64_t T_it;        /* reordering iterations (Algorithm 2)                               */
    int64_t s_b;         /* sum of the block ranks s_i = min(ceil(alpha n_i), m_i, n_i)       */
    int64_t s;           /* rank after the row update: min(ceil(alpha n1), s_b + m2, n1)      */
    int64_t r;           /* final rank: min(ceil(alpha min(m, n)), s + n2, m)                 */
} fastpi_split;

typedef struct {
    fastpi_precision precision;   /* FASTPI_FP64 (default) or FASTPI_MIXED                  */
    int max_sweeps;               /* Jacobi sweep cap (0 = default 60)                       */
    double tol;                   /* Jacobi rotation thresholds; 0 = defaults. The Jacobi    */
                                  /* block SVDs rotate columns of cosine above p * tol (p:   */
                                  /* block rows; default tol = eps of the block precision;   */
                                  /* the FP32 blocks of FASTPI_MIXED never go below FP32     */
                                  /* eps); every eigensolver (the cores of both updates, the */
                                  /* Gram route of large blocks, the randomized solver's     */
                                  /* small problems) above tol itself (default: its padded   */
                                  /* order * FP64 eps; 1e-8 for the Rayleigh-Ritz problems   */
                                  /* of FASTPI_MIXED's subspace core solver)                 */
    size_t max_workspace_bytes;   /* 0 = unlimited; larger needs fail with FASTPI_ENOMEM     */
} fastpi_options;

/* Schedule of the batched kernels (all values must be from the listed sets). */
typedef struct {
    int32_t block_lds;          /* LDS bytes of a block-SVD workgroup, 4096..61440; blocks whose  */
                                /* Jacobi state does not fit work in global scratch               */
    int32_t block_wgs_per_cu;   /* persistent block-SVD workgroups per compute unit, 1..16         */
    int32_t gram_rows;          /* rows of X per eigensolver partial-Gram workgroup: 64, 128, 256  */
    int32_t inner_sweeps;       /* Jacobi sweeps per 32 x 32 pair solve: 1 or 2                    */
    int32_t precond;            /* 1: run the core Jacobi on R^T of a pivoted Cholesky G = R^T R  */
                                /* (fewer sweeps); 0: on G itself                                 */
    int32_t eig_fused;          /* 1 (default): two launches per eigensolver round (the column    */
                                /* update fused with the next round's partial Grams, on two       */
                                /* iterates; the pair solves); 0: three launches per round on one */
                                /* iterate. Same results bitwise                                  */
} fastpi_tuning;

/*
 * Inner solver of the two incremental updates (Section 3.3). The paper computes the
 * update's truncated SVD exactly, or, for a low target rank, with a randomized method with
 * power iterations (oversampling 5 and 11 iterations in its experiments). Here the
 * randomized branch is subspace iteration on the update's Gram matrix G (order q, target
 * rank t): Y = G Omega with a Gaussian Omega of t + oversample columns, `iters` times an
 * orthonormalization of Y followed by Y = G Y, and the Rayleigh-Ritz eigenpairs of G on the
 * final basis. Omega comes from Philox4x32-10 with key (seed, update: 0 row, 1 column) and
 * counter = pair index (Box-Muller on two 53-bit uniforms per counter).
 *   mode: 0 = exact (default); 1 = randomized for an update with t < ceil(0.3 q);
 *         2 = randomized for every update with t + oversample < q.
 *   oversample in [0, 256], iters in [0, 64].
 */
typedef struct {
    int32_t mode;
    int32_t oversample;
    int32_t iters;
    uint32_t seed;
} fastpi_inner;

typedef struct fastpi_plan fastpi_plan;
typedef struct fastpi_handle fastpi_handle;
typedef struct fastpi_batch fastpi_batch;
typedef struct fastpi_labels fastpi_labels;

/* ceil(alpha * x) evaluated in IEEE double, clamped at 0 (Table 1: r = ceil(alpha n)). */
int64_t fastpi_target_rank(double alpha, int64_t x);

/*
 * Matrix reordering (Section 3.2, Algorithm 2). Host only, synchronous, integer work whose
 * result is bit-exact and independent of threads and platform.
 *   m, n         : shape of A (m, n >= 1)
 *   rowptr       : host int64[m+1], col: host int32[nnz]; CSR pattern, columns strictly
 *                  increasing in each row; val: host double[nnz] or NULL. When val is given,
 *                  stored zeros are not edges (Definition 1).
 *   k            : hub selection ratio, 0 < k < 1 (the paper uses 0.01)
 *   piT, piF     : host int32[m], int32[n] outputs: original row/column -> new row/column
 *   blocks       : host int64[4*blocks_cap] output (row0, col0, rows, cols) of every diagonal
 *                  block of A11 in new ids, in order; may be NULL when blocks_cap is 0
 *   num_blocks   : host output, the number of blocks (also when blocks_cap is too small,
 *                  which returns FASTPI_EINVAL after filling nothing)
 *   out          : host output shape report (the rank fields are 0: no alpha is involved)
 * Tie-breaks: hubs by (degree in the current graph descending, index ascending), the first
 * hub of a batch takes the highest free id; components discovered by scanning rows then
 * columns in ascending original index; the giant component is the largest (rows+columns),
 * first found on ties; non-giant components take the lowest free ids in discovery order,
 * rows then columns each ascending; the loop stops once the giant component has fewer rows
 * than this iteration's row-hub count or fewer columns than its column-hub count; the last
 * giant component becomes the last block.
 */
int fastpi_reorder(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col,
                   const double* val, double k, int32_t* piT, int32_t* piF,
                   int64_t* blocks, int64_t blocks_cap, int64_t* num_blocks, fastpi_split* out);

/*
 * The same reordering computed on the GPU of a handle (Section 3.2, Algorithm 2, with the
 * tie-breaks above; the result is identical to fastpi_reorder's). The CSR is in device
 * memory: rowptr int64[m+1], col int32[nnz], val double[nnz] or NULL; it is validated on
 * the device first (rowptr from 0 to nnz and monotone, columns in range and strictly
 * increasing within a row, finite values), with the error codes of fastpi_reorder. The
 * outputs are host buffers as in fastpi_reorder. Synchronous on the handle's stream.
 */
int fastpi_reorder_gpu(fastpi_handle* h, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                       const int32_t* col, const double* val, double k, int32_t* piT, int32_t* piF,
                       int64_t* blocks, int64_t blocks_cap, int64_t* num_blocks, fastpi_split* out);

/*
 * Plan for one sparsity pattern and one alpha (Algorithm 1, line 1, plus the rank rule
 * of Eqs. 1-3): runs the reordering, derives every block's rank, and precomputes the index
 * maps that move values from the caller's CSR into the blocks of A11, A21 and T = [A12; A22].
 * Host only and synchronous. The CSR arguments are as in fastpi_reorder; the plan keeps no
 * pointer to them. alpha in (0, 1], 0 < k < 1.
 */
int fastpi_plan_create(fastpi_plan** plan, int64_t m, int64_t n, const int64_t* rowptr,
                       const int32_t* col, const double* val, double alpha, double k);
/* As fastpi_plan_create (host CSR, validated on the host), with the reordering run on the
 * handle's GPU (fastpi_reorder_gpu); the plan is the same. */
int fastpi_plan_create_gpu(fastpi_plan** plan, fastpi_handle* h, int64_t m, int64_t n,
                           const int64_t* rowptr, const int32_t* col, const double* val,
                           double alpha, double k);
int fastpi_plan_info(const fastpi_plan* plan, fastpi_split* out);
/* Copies the permutations (host int32[m], int32[n]); either pointer may be NULL. */
int fastpi_plan_permutation(const fastpi_plan* plan, int32_t* piT, int32_t* piF);
/* Copies the block table, host int64[4*B], (row0, col0, rows, cols) per block. */
int fastpi_plan_blocks(const fastpi_plan* plan, int64_t* blocks);
/* Copies the rank s_i of every block (host int64[B]). */
int fastpi_plan_block_ranks(const fastpi_plan* plan, int64_t* ranks);
void fastpi_plan_destroy(fastpi_plan* plan);

/*
 * The 16 features of every dense diagonal block (height and width > 0), in block order, as
 * rows of out (host double[B_dense * 16]); val is the caller's host CSR values (the plan's
 * pattern). Features: log rows, log cols, log nnz, density, log ||A_i||_F^2, log max / log min
 * / mean / std of the log squared column norms (in that order: max, min, mean, std),
 * log max squared row norm, ||A_i||_F^2 / max squared column norm, the block's share of
 * ||A11||_F^2, alpha, cols / n1, log(1 + edges from the block into hub rows and columns),
 * block index / number of blocks. Used by the learned rank predictor.
 */
int fastpi_block_features(const fastpi_plan* plan, const double* val, double* out);

/*
 * Replaces the per-block ranks of Eq. 1 (host int64[B], one per block, 0 for blocks of height
 * or width 0) and recomputes s_b, s and r; each rank is clamped to min(rows, cols). Lets a
 * learned allocation replace the ceil(alpha n_i) rule. Upload the plan again afterwards.
 */
int fastpi_plan_set_block_ranks(fastpi_plan* plan, const int64_t* ranks);

/*
 * Learned allocation of the block ranks: the learned form of Eq. 1's rank rule
 * (s_i = ceil(alpha n_i) per diagonal block), with the same total s_b.
 *   fastpi_rank_model: the training statistics of the 16 block features (fastpi_block_features
 *     order), each host double[16]: mean, std (every entry > 0), lo and hi (the minimum and
 *     maximum over the training set); margin >= 0: a block is in range when every feature f_j
 *     lies in [lo_j - margin span_j, hi_j + margin span_j], span_j = max(hi_j - lo_j, 1e-12).
 *   fastpi_rank_inputs: for n feature rows (host double[n*16]), the network's input
 *     X = (f - mean) / std rounded to float (host float[n*16]) and the range flags (host
 *     int32[n], 1 = in range); either output may be NULL. Host only.
 *   fastpi_rank_allocate: integer ranks s (host int64[n]) with 0 <= s_i <= q_i and sum exactly
 *     min(budget, sum q_i), in proportion to x_i = max(f_i q_i, 1e-9), f_i (host float[n])
 *     clipped to [0, 1] (NaN read as 0), q (host int64[n]) >= 0: the largest scale c with
 *     sum_i min(c x_i, q_i) <= budget is located by 200 bisection steps on
 *     [0, max q / min x + 1] (sums in index order), s_i = floor(min(c x_i, q_i)), and the
 *     units still missing go one each to the blocks with the largest fractional parts (ties to
 *     the lower index) that are below q_i. Host only.
 *   fastpi_plan_learned_ranks: the whole allocation for the plan, written to ranks (host
 *     int64[B], block order, 0 for blocks of height or width 0); val is the host CSR values of
 *     the plan's pattern. Out-of-range blocks keep the alpha rule's rank
 *     min(ceil(alpha cols), rows, cols); the network (theta: device float[5313], the packed
 *     parameters below) runs on the handle's GPU for the in-range blocks, which share the alpha
 *     rule's total s_b minus the out-of-range ranks through fastpi_rank_allocate with
 *     q_i = min(rows, cols). The plan is not changed (apply the result with
 *     fastpi_plan_set_block_ranks). Synchronises the handle's stream; allocates and frees
 *     device memory for the network's input and output.
 * Errors: FASTPI_EINVAL for null pointers, n < 0, a std entry <= 0 or a negative margin or q_i;
 * FASTPI_ENOMEM / FASTPI_EHIP from the device part.
 */
typedef struct fastpi_rank_model {
    const double* mean;
    const double* std;
    const double* lo;
    const double* hi;
    double margin;
} fastpi_rank_model;
int fastpi_rank_inputs(int64_t n, const double* feats, const fastpi_rank_model* model, float* X,
                       int32_t* in_range);
int fastpi_rank_allocate(int64_t n, const float* f, const int64_t* q, int64_t budget, int64_t* s);
int fastpi_plan_learned_ranks(const fastpi_plan* plan, fastpi_handle* h, const double* val,
                              const fastpi_rank_model* model, const float* theta, int64_t* ranks);

/*
 * Learned rank predictor: a 16-64-64-1 network (ReLU, ReLU, sigmoid), FP32, predicting a
 * block's kept fraction s_i / min(rows, cols). Packed parameters (device float[5313]):
 * W1 (64x16 row-major), b1 (64), W2 (64x64), b2 (64), W3 (64), b3.
 *   fastpi_mlp_forward : f = net(X) for X device float[N*16] (row-major), f device float[N];
 *   fastpi_mlp_gradient: gradient of mean((f - y)^2) over the N samples, grad device
 *                        float[5313], summed in a fixed order (bitwise reproducible);
 *   fastpi_mlp_adam    : one Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1)
 *                        on theta, with moment buffers m, v (device float[5313], start at 0).
 */
int fastpi_mlp_param_count(void);
int fastpi_mlp_forward(fastpi_handle* h, int64_t N, const float* X, const float* theta, float* f);
int fastpi_mlp_gradient(fastpi_handle* h, int64_t N, const float* X, const float* y,
                        const float* theta, float* grad);
int fastpi_mlp_adam(fastpi_handle* h, float* theta, const float* grad, float* m, float* v,
                    int64_t step, float lr);

/*
 * Device handle: binds a HIP device and stream (stream may be NULL for the default stream)
 * and owns the device workspace. opts may be NULL for the defaults.
 */
int fastpi_create(fastpi_handle** h, int device, void* hip_stream, const fastpi_options* opts);
int fastpi_set_precision(fastpi_handle* h, fastpi_precision p);
void fastpi_destroy(fastpi_handle* h);

/*
 * Copies the plan's tables to the handle's device (stream-ordered). Needed once per plan
 * before fastpi_svd; uploading another plan replaces it.
 */
int fastpi_upload_plan(fastpi_handle* h, const fastpi_plan* plan);

/*
 * Low-rank SVD A ~= U diag(S) V^T of the uploaded plan's matrix (Algorithm 1, lines 2-4:
 * block SVDs of A11 by Eq. 1, row update by Eq. 2, column update by Eq. 3), mapped back to
 * the caller's original row and column order.
 *   rowptr, col, val : device CSR of A, the same pattern the plan was built from
 *                      (int64[m+1], int32[nnz], double[nnz])
 *   U : device double[m * r] row-major;  S : device double[r], descending;
 *   V : device double[n * r] row-major;  r = fastpi_split.r of the plan.
 * The two updates and the diagonal blocks on the Gram route (blocks with p q^2 above the
 * route threshold) take their truncated factors from the eigenpairs of an FP64 Gram matrix,
 * which resolves a singular value only down to about sqrt(q eps) of the largest: every
 * singular value at or below 1e-7 * (the largest of its stage) is returned as exactly 0 with
 * its U column zero (and the V column unspecified), and fastpi_apply's S^+ is 0 there. When
 * that happens to a non-zero matrix, fastpi_sync returns FASTPI_WFLOOR (for an exactly
 * rank-deficient A this is expected: its zero singular values are at that floor). A with
 * singular values in (about 1e-12, 1e-7) times the largest therefore does not reach
 * Problem 1's exact pseudoinverse at alpha = 1; the truncated pseudoinverse it gives drops
 * those directions. Columns at or below max(m, n) * eps * S[0] carry no information either.
 * The two incremental cores are solved by Jacobi sweeps whose number depends on the data:
 * the host reads each sweep's convergence state (one sweep behind, on a side stream), so
 * the call returns once the last sweep is queued; the final stages are queued, not finished.
 */
int fastpi_svd(fastpi_handle* h, const int64_t* rowptr, const int32_t* col, const double* val,
               double* U, double* S, double* V);

/*
 * Pseudoinverse apply (Problem 1, Application 1): Z = V diag(S^+) U^T Y, with
 * S^+_i = 1/S_i when S_i > max(m, n) * eps * max(S), else 0.
 *   U : device double[m*r], S : device double[r], V : device double[n*r], row-major;
 *   Y : device double[m*L] row-major; Z : device double[n*L] row-major output.
 */
int fastpi_apply(fastpi_handle* h, int64_t m, int64_t n, int64_t r, const double* U,
                 const double* S, const double* V, int64_t L, const double* Y, double* Z);

/*
 * fastpi_apply without any device allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc). Same arguments,
 * layout and result as fastpi_apply; the intermediate S^+, U^T Y and its split-K partials
 * live in a fixed scratch of 8,388,608 doubles (64 MiB) that the library holds on every GPU
 * it runs on until the process ends. Needs r + 2 r L doubles at least (FASTPI_EINVAL
 * beyond that); when fastpi_apply's split of U^T Y does not fit, fewer splits are used (the
 * same result up to the summation order). Every call on a GPU shares that GPU's scratch:
 * calls that overlap on one GPU (two streams, two threads) race and must be serialised by
 * the caller.
 */
int fastpi_apply_noalloc(fastpi_handle* h, int64_t m, int64_t n, int64_t r, const double* U,
                         const double* S, const double* V, int64_t L, const double* Y, double* Z);

/*
 * Sparse label matrix of Application 1 (each row of Y is a binary label vector with few
 * positives). Y (m x L) is given as a host CSR: rowptr int64[m+1] (rowptr[0] = 0, monotone),
 * col int32[nnz] in [0, L), val double[nnz] or NULL for all ones. The object keeps a device
 * copy of Y^T (per label, its rows in increasing order) and the work split used by
 * fastpi_apply_sparse; the host arrays may be freed when the call returns (it waits for the
 * copies on the handle's stream). Errors: FASTPI_EINVAL for a malformed pattern,
 * FASTPI_ENONFINITE for a non-finite value, FASTPI_ENOMEM.
 */
int fastpi_labels_create(fastpi_labels** y, fastpi_handle* h, int64_t m, int64_t L,
                         const int64_t* rowptr, const int32_t* col, const double* val);
void fastpi_labels_destroy(fastpi_labels* y);
int fastpi_labels_nnz(const fastpi_labels* y, int64_t* nnz);

/*
 * Pseudoinverse apply with a sparse Y (Application 1, Problem 1):
 * Z = V diag(S^+) U^T Y, S^+ as in fastpi_apply. U^T Y is formed as Y^T U over Y's
 * positives only (cost proportional to nnz(Y) * r rather than m * L * r), in a fixed
 * summation order, then Z = V (Y^T U diag(S^+))^T.
 *   U : device double[m*r], S : device double[r], V : device double[n*r], row-major;
 *   Y : labels created on this handle's device with m rows;
 *   Z : device double[n*L] row-major output (zero when r = 0).
 */
int fastpi_apply_sparse(fastpi_handle* h, int64_t m, int64_t n, int64_t r, const double* U,
                        const double* S, const double* V, const fastpi_labels* Y, double* Z);

/*
 * Top-k precision counts of the accuracy experiment (Section 4) on held-out rows. For each
 * row x of a device CSR test matrix (rows x n: rowptr int64[rows+1], col int32, val double),
 * the score vector yhat = Z^T x (Z: device double[n*L] row-major) is accumulated over x's
 * entries in storage order, one rounded multiply and one rounded add per entry; labels are
 * ranked by descending score, equal scores to the lower label, non-finite scores never.
 * hits[row * nk + t] (device int32[rows*nk]) = number of positives of the row (device CSR
 * y_rowptr int64[rows+1], y_col int32) among its ks[t] top-ranked labels; P@k of the set is
 * sum over rows of hits / (rows * k). ks is a host array of nk (1..16) values in [1, 64].
 * A row with a column outside [0, n) gets -1 counts. The CSR arrays must be well formed
 * (the kernel reads rowptr[0..rows] and the entries they address).
 */
int fastpi_topk_hits(fastpi_handle* h, int64_t rows, int64_t n, int64_t L, const int64_t* rowptr,
                     const int32_t* col, const double* val, const double* Z, const int64_t* y_rowptr,
                     const int32_t* y_col, int32_t nk, const int32_t* ks, int32_t* hits);

/*
 * Intermediate results of the last fastpi_svd on this handle, for stage-level checks.
 * which: 0 = block singular values sigma1 (s_b, block order, each block descending),
 *        1 = row-update singular values sigma2 (s), 2 = row-update right factor V2 (n1 x s,
 *        reordered column ids), 3 = row-update left factor U2 (m x s, reordered row ids).
 * dst is a device pointer with room for count doubles; count must equal the stage's size.
 */
int fastpi_stage_output(fastpi_handle* h, int which, double* dst, int64_t count);

/*
 * Dense symmetric eigensolver used for the incremental cores (FP64 block Jacobi, started
 * from a pivoted Cholesky factor of G unless the handle's schedule sets precond = 0).
 *   q    : order; G : device double[q*q] (symmetric, read only);
 *   t    : number of leading eigenpairs wanted (0 < t <= q);
 *   vals : device double[t], descending; vecs : device double[q*t] row-major, column k is
 *          the eigenvector of vals[k].
 */
int fastpi_syev_top(fastpi_handle* h, int64_t q, const double* G, int64_t t, double* vals,
                    double* vecs);

/*
 * Stage-level check of the matrix-core product used by the dense steps (the subspace core
 * solver's products, the update and apply GEMMs): C = op(A) op(B) on the handle's stream,
 * op(A) = A (M x K, lda) or, with ta, A stored K x M; op(B) = B (K x N, ldb) or, with tb,
 * B stored N x K; all device FP64 row-major; fp32 = 1 rounds the operands to FP32 and
 * accumulates in FP32 (the mixed form). Any shape is accepted (the kernel masks the edges).
 */
int fastpi_mfma_gemm(fastpi_handle* h, int ta, int tb, int64_t M, int64_t N, int64_t K, const double* A,
                     int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc, int fp32);

/* Waits for the handle's stream and reports device-side failures of the last fastpi_svd
 * (FASTPI_ENONFINITE: non-finite input; FASTPI_ENOCONV: a Jacobi sweep cap reached), or the
 * warning FASTPI_WFLOOR (a kept singular value under the Gram floor, see fastpi_svd). */
int fastpi_sync(fastpi_handle* h);

/* Number of sweeps used by the last Jacobi run of each kind on this handle:
 * out[0] = block stage (max over blocks), out[1] = row-update core, out[2] = column-update core. */
int fastpi_last_sweeps(fastpi_handle* h, int32_t* out3);

/*
 * Pairs of 16-column blocks whose 32 x 32 Jacobi solve ran (rather than being found
 * orthogonal already) in the last fastpi_svd: out2[0] row-update core, out2[1] column-update
 * core (the work count behind the eigensolver's algorithmic flops).
 */
int fastpi_last_rotations(fastpi_handle* h, int64_t* out2);

/*
 * Measurement hook: times every launch of one kernel of the device path with a HIP event
 * pair on the handle's stream (each timed launch costs an extra event record).
 * kind: 0 = eigensolver partial Gram, 1 = eigensolver pair solve, 2 = eigensolver column
 * update, 3 = block SVD launches, 4 = the label SpMM of fastpi_apply_sparse (both passes),
 * 5 = fastpi_topk_hits, 6 = the transposed-B GEMM of fastpi_apply_sparse, 7 = the products by G
 * of the subspace core solver (fastpi_set_core_solver), 8 = its Cholesky-QR panel kernel,
 * 9 = the eigensolver's fused column update and partial Grams (fastpi_tuning.eig_fused = 1,
 * the default; kinds 0 and 2 then time nothing), -1 = off.
 * Starting discards earlier timings.
 */
int fastpi_timing_start(fastpi_handle* h, int kind);
/* Waits for the stream; returns the number of timed launches and their summed duration in
 * milliseconds since fastpi_timing_start, and clears them (timing stays on). */
int fastpi_timing_read(fastpi_handle* h, int64_t* launches, double* total_ms);

/*
 * Graph mode (batching form of the path): when enabled, fastpi_svd replays HIP graphs of
 * the stage chain instead of launching each kernel -- one graph for the stages before,
 * between and after the two eigensolvers and one per eigensolver sweep, since the number
 * of sweeps is data dependent. The graphs are captured on the first call and captured
 * again whenever a pointer, the precision or a Jacobi option changes. The results are
 * bitwise identical to the eager launches. Kernel timing (fastpi_timing_*) sees eager runs
 * only.
 */
int fastpi_set_graph(fastpi_handle* h, int enable);
/* Graph launches of the last fastpi_svd (0 for an eager run, -1 for a null handle). */
int64_t fastpi_last_graph_launches(const fastpi_handle* h);

/* Schedule of the handle's batched kernels (the defaults, or what the autotuner chose). */
int fastpi_set_tuning(fastpi_handle* h, const fastpi_tuning* t);
int fastpi_get_tuning(const fastpi_handle* h, fastpi_tuning* t);
/*
 * Tuning cache: a text file of "key|block_lds wgs_per_cu gram_rows inner_sweeps precond" lines, the
 * key naming the GPU architecture, the precision and the shape bucket (log2 of the number
 * of matrices, of blocks and of the two core orders). Plans uploaded (and batches created)
 * afterwards take a matching entry; fastpi_autotune reads and writes it. NULL clears it.
 */
int fastpi_set_tuning_cache(fastpi_handle* h, const char* path);

/*
 * Route of the diagonal blocks of A11 (Eq. 1). A block whose sides p >= q give
 * p * q^2 < min_cost is solved by one workgroup's one-sided Jacobi (the persistent block
 * launch); a costlier one through the Gram matrix of its long side: G = X^T X (q x q), the
 * batched FP64 eigensolver of the updates, and the other factor X E diag(sigma^-1)
 * (singular values below 1e-7 of the block's largest are returned as zero). Default 1e6;
 * 0 sends every block with rank > 0 and q >= 2 that way. Kept across fastpi_upload_plan; a
 * batch takes the handle's setting when it is created.
 */
int fastpi_set_block_route(fastpi_handle* h, double min_cost);
int fastpi_batch_set_block_route(fastpi_batch* b, double min_cost);

/*
 * Core solver of the exact branch (the truncated SVD of M2 and of X3, Eqs. 2-3, taken as the
 * top t eigenpairs of their Gram matrix G of order q). mode 0: block one-sided Jacobi on G
 * for every core. mode 1 (default): where q >= min_order and k = 32 * ceil(f * t / 32) is at
 * most max_frac * q (f = k_factor in FASTPI_FP64, k_factor_mixed in FASTPI_MIXED: a smaller
 * basis needs more products for the same accuracy, and the mixed form's gates are looser),
 * subspace iteration with a k-column block: products Y = G Q (FP32
 * in FASTPI_MIXED), a Cholesky QR of the block before every orth_every-th product, a fixed
 * number of products (iters_fp64, iters_mixed), two FP64 Cholesky QRs, then Rayleigh-Ritz:
 * the top t eigenpairs of Q^T G Q by the block Jacobi, vectors Q W. Every such core is
 * checked (each pair's residual ||G v - lambda v|| against res_tol * lambda_1 of the form,
 * the rank of every Cholesky QR); a core that fails is solved again by Jacobi on G, so the
 * result is always the converged one. Ranges: min_order >= 64, 1 <= k_factor, k_factor_mixed <= 8,
 * 0 < max_frac <= 1, iterations 1..256, orth_every 1..4, tolerances > 0.
 */
typedef struct {
    int32_t mode;
    int32_t min_order;
    double k_factor;
    double max_frac;
    int32_t iters_fp64;
    int32_t iters_mixed;
    int32_t orth_every;
    int32_t pad;
    double res_tol_fp64;
    double res_tol_mixed;
    double k_factor_mixed;
} fastpi_core_solver;
/* Kept across fastpi_upload_plan; a batch takes the handle's setting when it is created. */
int fastpi_set_core_solver(fastpi_handle* h, const fastpi_core_solver* c);
int fastpi_get_core_solver(const fastpi_handle* h, fastpi_core_solver* c);
int fastpi_batch_set_core_solver(fastpi_batch* b, const fastpi_core_solver* c);
/* Route each core took in the last fastpi_svd (out2[0] row update, out2[1] column update) or
 * batch run (out: 2 per matrix): 0 Jacobi, 1 subspace iteration, 2 subspace iteration that
 * failed its check and was solved again by Jacobi, 3 the randomized branch. */
int fastpi_last_core_routes(const fastpi_handle* h, int32_t* out2);
int fastpi_batch_core_routes(const fastpi_batch* b, int32_t* out);

/* Selects the inner solver of the handle's runs (kept across fastpi_upload_plan; a batch
 * takes the handle's setting when it is created). FASTPI_EINVAL for values out of range. */
int fastpi_set_inner(fastpi_handle* h, const fastpi_inner* c);
int fastpi_get_inner(const fastpi_handle* h, fastpi_inner* c);
int fastpi_batch_set_inner(fastpi_batch* b, const fastpi_inner* c);
/* 1 when the setting takes the randomized branch for an update of target rank t and
 * order q, else 0. */
int fastpi_inner_applies(const fastpi_inner* c, int64_t t, int64_t q);
/* Stage-level check of the test-matrix generator: out[0..count) (device) = the standard
 * normals the randomized branch draws for key (seed, stream), in row-major element order. */
int fastpi_gaussian(fastpi_handle* h, int64_t count, uint32_t seed, uint32_t stream, double* out);
/*
 * Autotuner: runs the uploaded plan's path with every candidate schedule (three block-SVD
 * LDS/occupancy pairs timed on the block launch alone, then six eigensolver schedules --
 * partial-Gram height, inner sweeps, preconditioner -- timed over whole runs), keeps the fastest and stores it in the tuning cache when one is set.
 * Arguments as for fastpi_svd (the outputs hold a valid result afterwards). report, when
 * not NULL, receives a one-line summary of the timings (truncated to report_cap bytes).
 * Synchronous. A cache hit skips the trials.
 */
int fastpi_autotune(fastpi_handle* h, const double* val, double* U, double* S, double* V,
                    char* report, int64_t report_cap);

/*
 * Batches: several independent matrices that run together on the handle's device and
 * stream. Every diagonal block of every matrix goes through one persistent block-SVD launch
 * (an atomic work queue, largest blocks first), the row-update and the column-update cores
 * of all matrices through one batched eigensolver each (one launch per kernel and round for
 * all matrices), and the other stages per matrix. The batch keeps its own device copy of
 * every plan; the plans may be destroyed afterwards. The handle must outlive the batch.
 */
int fastpi_batch_create(fastpi_batch** b, fastpi_handle* h, int64_t count,
                        const fastpi_plan* const* plans);
void fastpi_batch_destroy(fastpi_batch* b);
/*
 * fastpi_svd for every matrix of the batch. val, U, S, V are HOST arrays of count DEVICE
 * pointers, laid out per matrix as in fastpi_svd. Uses the handle's precision and options.
 */
int fastpi_batch_svd(fastpi_batch* b, const double* const* val, double* const* U,
                     double* const* S, double* const* V);
/*
 * Waits for the stream. status (host int32[count], may be NULL) receives each matrix's own
 * fastpi_status, so that one failing matrix (e.g. a non-finite value) leaves the others'
 * results and codes intact; sweeps (host int32[3*count], may be NULL) the sweep counts as
 * in fastpi_last_sweeps. Returns the first negative (error) code, else FASTPI_WFLOOR if any
 * matrix has that warning, else FASTPI_OK.
 */
int fastpi_batch_sync(fastpi_batch* b, int32_t* status, int32_t* sweeps);
/* fastpi_last_rotations for every matrix of the batch: out[2*i], out[2*i+1] (host int64). */
int fastpi_batch_rotations(const fastpi_batch* b, int64_t* out);
int fastpi_batch_set_graph(fastpi_batch* b, int enable);
int64_t fastpi_batch_last_graph_launches(const fastpi_batch* b);
int fastpi_batch_set_tuning(fastpi_batch* b, const fastpi_tuning* t);
int fastpi_batch_get_tuning(const fastpi_batch* b, fastpi_tuning* t);
int fastpi_batch_autotune(fastpi_batch* b, const double* const* val, double* const* U,
                          double* const* S, double* const* V, char* report, int64_t report_cap);

const char* fastpi_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FASTPI_H */
