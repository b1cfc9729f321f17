// Device-side driver of the path: per-matrix device plans and workspaces ("instances") and
// the group runner that takes any number of instances through the stages together.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "host_internal.h"
#include "kernels.h"

namespace fastpi {

// Schedule parameters of the batched kernels (chosen by the autotuner, or defaults).
struct Tuning {
    int block_lds = 32 * 1024;   // dynamic LDS bytes of a block-SVD workgroup
    int block_wgs_per_cu = 4;    // persistent block-SVD workgroups per compute unit
    int gram_rows = 128;         // rows per partial-Gram workgroup in the eigensolver
    int inner_sweeps = 1;        // inner Jacobi sweeps per pair solve
    int precond = 1;             // pivoted-Cholesky start of the core eigensolvers
    int core_mode = -1;          // core solver route chosen by the autotuner (-1: the group's own)
    int eig_fused = 1;           // eigensolver rounds in two launches (0: three launches a round)
};
bool tuning_valid(const Tuning& t);

// Inner solver of the two incremental updates (Section 3.3): exact truncated SVD, or
// randomized subspace iteration on the update's Gram matrix for a low target rank.
struct InnerCfg {
    int mode = 0;         // 0 exact; 1 randomized where t < ceil(0.3 q); 2 wherever t + oversample < q
    int oversample = 5;
    int iters = 11;
    uint32_t seed = 0;
};
bool inner_valid(const InnerCfg& c);
bool inner_applies(const InnerCfg& c, int64_t t, int64_t q);

// A diagonal block of A11 too costly for one workgroup's one-sided Jacobi (p q^2 at least
// kBigBlockCost, p >= q its sides): its SVD goes through the Gram matrix of its long side,
// G = X^T X (q x q), the batched FP64 eigensolver, and W = X E for the other factor.
constexpr double kBigBlockCost = 1.0e6;
struct BigBlock {
    int inst = 0;                // index of its matrix in the group
    const double* A = nullptr;   // dense block, column-major rows x cols
    double *U = nullptr, *V = nullptr, *sig = nullptr;   // the block's packed outputs
    int64_t rows = 0, cols = 0, p = 0, q = 0, t = 0;
    bool trans = false;          // rows < cols: X = A^T
    double *G = nullptr, *E = nullptr, *lam = nullptr, *W = nullptr, *part = nullptr;
    int sp = 1;        // K split of the transposed products (the Gram when trans, W otherwise)
    int sp_nt = 1;     // K split of the Gram X X^T when not trans (a small q over a long p)
};

// One randomized core: the top t eigenpairs of a q x q Gram matrix G from a k-dimensional
// basis (k = t + oversample), written where the exact solver would write them.
struct RandCore {
    int inst = 0;
    int64_t q = 0, t = 0, k = 0;
    const double* G = nullptr;
    double *Y = nullptr, *Q = nullptr, *W = nullptr, *Wv = nullptr, *Ws = nullptr, *Wd = nullptr,
           *part = nullptr;
    int sp = 1;
    double* lam_out = nullptr;
    double* vec_out = nullptr;
    int32_t sweeps = 0;     // Jacobi sweeps over all eigensolves of the last run
    int64_t rotated = 0;
};

// Core solver of the two updates' exact branch: the existing block Jacobi on G, or subspace
// iteration (Y = G Q with Cholesky-QR orthonormalisation every `orth_every` products, a
// fixed number of products, a final double orthonormalisation and Rayleigh-Ritz through the
// block Jacobi of the k x k projected matrix) where the basis k = ceil32(k_factor t) is small
// against q (its own factor per precision form). Each result is checked (residual of every kept pair against res_tol * lambda_1,
// rank of every orthonormalisation); a core that fails the check is solved again by Jacobi.
struct CoreCfg {
    int mode = 1;             // 0: Jacobi for every core; 1: subspace iteration where it applies
    int min_order = 1024;     // cores of smaller order stay on Jacobi
    double k_factor = 2.0;    // basis factor of the FP64 form
    double max_frac = 0.65;   // and k <= max_frac * q
    int iters_fp64 = 28;      // products by G (FP64 form)
    int iters_mixed = 18;     // products by G in FP32 (mixed form)
    int orth_every = 2;
    double res_tol_fp64 = 1e-9;
    double res_tol_mixed = 1e-5;
    double k_factor_mixed = 1.5;   // basis factor of the mixed form
    double rr_tol_mixed = 1e-8;    // cosine threshold of the Rayleigh-Ritz Jacobi, mixed form
};
bool core_cfg_valid(const CoreCfg& c);
// basis size of the subspace route for target t and order q in the given precision form, or 0
// when the core stays on Jacobi
int64_t core_basis(const CoreCfg& c, int64_t t, int64_t q, bool mixed);

// One core on the subspace route (buffers in one allocation per core).
struct SubCore {
    int inst = 0;
    int64_t q = 0, t = 0, k = 0;
    int kp = 0, sp = 1;
    int gsplit = 1;             // K split of the products by G (partials in gpart)
    const double* G = nullptr;
    double *Q = nullptr, *Y = nullptr, *H = nullptr, *Wv = nullptr, *part = nullptr, *gpart = nullptr;
    double* lam_out = nullptr;
    double* vec_out = nullptr;
};
struct SubSet {
    std::vector<SubCore> cores;
    std::vector<CholJob> chol;      // host copy of the Cholesky-QR job table
    CholJob* dchol = nullptr;
    int* flags = nullptr;           // device, one per core
    int* host_flags = nullptr;      // pinned
    int max_kp = 0;
    // the k x k Rayleigh-Ritz matrices are jobs of the update's batched Jacobi set (set2 or
    // set3), next to the cores that stay on Jacobi, so that one eigensolve serves both
    EigSet fb;                      // block Jacobi on G itself, for cores that fail the check
    std::vector<void*> allocs;
    int fallbacks = 0;              // cores solved again by Jacobi in the last run
    bool basis_in_q = true;         // after the pre-phase: the basis is in Q (else in Y)
};

struct DevicePlan {
    bool valid = false;
    int64_t m = 0, n = 0, nnz = 0, m1 = 0, n1 = 0, m2 = 0, n2 = 0, s_b = 0, s = 0, r = 0;
    int64_t B_dense = 0, val_elems = 0, blk_elems = 0, u1 = 0, v1 = 0;
    int64_t off_a21r = 0, off_a21c = 0, off_tr = 0, off_tc = 0;
    BlockWork* work = nullptr;
    int64_t *dst0 = nullptr, *dst1 = nullptr;
    int64_t *a21_rowptr = nullptr, *a21_colptr = nullptr, *t_rowptr = nullptr, *t_colptr = nullptr;
    int *a21_colidx = nullptr, *a21_rowidx = nullptr, *t_colidx = nullptr, *t_rowidx = nullptr;
    int *piT = nullptr, *invT = nullptr, *invF = nullptr;
    SegDev seg_a21c{}, seg_a21r{}, seg_tc{}, seg_tr{};
};

// One matrix: its device plan, workspace and status words.
struct Instance {
    DevicePlan dp;
    std::vector<void*> allocs;          // device plan tables
    std::vector<BlockWork> work;        // host copy of the block work list
    std::vector<int64_t> scratch_off;   // per work item, in doubles, inside the scratch region
    double* ws = nullptr;
    size_t ws_bytes = 0;
    int* iws = nullptr;
    size_t iws_bytes = 0;
    int* status = nullptr;   // device [0] status bits, [1] block sweeps (not owned)
    int32_t sweeps[3] = {0, 0, 0};
    int64_t rotated[2] = {0, 0};   // pairs rotated by the row- and column-update eigensolvers
    int32_t route[2] = {0, 0};     // core route of the last run: 0 Jacobi, 1 subspace, 2 subspace
                                   // then Jacobi (failed check), 3 randomized
    // offsets (in doubles) of the stage buffers inside ws
    int64_t o_vals = 0, o_u1 = 0, o_v1 = 0, o_sig1 = 0, o_g2 = 0, o_v2 = 0, o_lam2 = 0, o_sig2 = 0,
            o_inv2 = 0, o_u2 = 0, o_g3 = 0, o_vt = 0, o_lam3 = 0, o_sig3 = 0, o_inv3 = 0, o_c1 = 0,
            o_c2 = 0, o_eig = 0, o_part = 0, o_gs = 0, o_spart = 0, o_end = 0;
};

// Uploads the plan's tables and sizes the workspace (cap: 0 = none). Synchronises `st`.
int instance_upload(Instance& I, const Plan& p, size_t ws_cap, hipStream_t st);
// Copies a segment table to the device; every allocation is appended to `allocs`.
int upload_segments(std::vector<void*>& allocs, const Segments& s, SegDev& d, hipStream_t st);
void instance_free(Instance& I, hipStream_t st);

struct RunCfg {
    hipStream_t st = nullptr;
    hipStream_t copy_st = nullptr;
    KernelTimer* timer = nullptr;   // eager runs only
    bool mixed = false;
    int max_sweeps = 60;
    double tol = 0;
    bool use_graph = false;
};

// A set of instances that run together: one persistent block-SVD launch over all their
// blocks, one batched eigensolver per update step, and the remaining stages per instance.
struct Group {
    std::vector<Instance*> inst;
    int ncu = 256;
    Tuning tune;
    BlockTask* tasks = nullptr;
    int ntasks = 0;
    int* counter = nullptr;
    double big_cost = kBigBlockCost;   // p q^2 from which a block takes the Gram route
    double eig_tol = 0;                // cosine threshold of every eigensolver job (0: order * eps)
    std::vector<BigBlock> big;      // blocks on the Gram route (not in `tasks`)
    EigSet set1;                    // their eigensolves
    std::vector<void*> ballocs;
    EigSet set2, set3;              // exact cores
    InnerCfg inner;
    std::vector<RandCore> rcores[2];   // randomized cores of the row and column updates
    std::vector<char> sign_v2;         // per instance: fix the signs of V2 (randomized column update)
    EigSet rset[2];                    // their k x k eigensolves
    std::vector<void*> rallocs;
    CoreCfg core;
    bool mixed = false;                // precision form the core sets are built for (the basis
                                       // of the subspace route depends on it)
    SubSet sub[2];                     // cores of the row and column updates on the subspace route
    // captured graphs: stages before, between and after the two eigensolvers, and one
    // sweep of each eigensolver
    hipStream_t cap = nullptr;
    hipGraphExec_t g_front = nullptr, g_sw1 = nullptr, g_front2 = nullptr, g_sw2 = nullptr, g_mid = nullptr,
                   g_sw3 = nullptr, g_back = nullptr;
    std::vector<uint64_t> key;
    int graph_launches = 0;   // graph launches of the last run
};

int group_build(Group& g, int device, hipStream_t st);
void group_free(Group& g);
void group_drop_graphs(Group& g);
int group_set_tuning(Group& g, const Tuning& t, hipStream_t st);
int group_set_inner(Group& g, const InnerCfg& c, hipStream_t st);
int group_set_core(Group& g, const CoreCfg& c, hipStream_t st);
// Computes U, S, V of every instance (arrays of device pointers, one per instance).
int group_svd(Group& g, const double* const* val, double* const* U, double* const* S,
              double* const* V, const RunCfg& c);

// Autotuner: times the candidate schedules on the group's own data and keeps the fastest.
// The result is stored in (and first looked up from) a text cache keyed by the device
// architecture, the precision and the shape bucket of the group, when `cache` is not null.
int group_autotune(Group& g, const double* const* val, double* const* U, double* const* S,
                   double* const* V, const RunCfg& c, const char* cache, int device,
                   std::string* report);
int tuning_lookup(const Group& g, const char* cache, int device, bool mixed, Tuning& out);

}  // namespace fastpi
