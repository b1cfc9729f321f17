// Device-side driver: instance upload, the staged run of a group of instances (eager or
// from captured graphs) and the autotuner of the batched kernels' schedules.
#include "driver.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <fstream>
#include <sstream>

namespace fastpi {

namespace {

#define HIP_TRY(expr)                                                               \
    do {                                                                            \
        hipError_t _e = (expr);                                                     \
        if (_e != hipSuccess) {                                                     \
            set_error(std::string("HIP error: ") + hipGetErrorString(_e) + " at " + \
                      #expr);                                                       \
            return FASTPI_EHIP;                                                     \
        }                                                                           \
    } while (0)

// Singular values at or below this fraction of the largest are not resolved by the Gram
// route (about sqrt(q eps)); they are returned as zero and the matrix's status word takes
// the floor warning bit.
constexpr double kRelCut = 1e-7;
// Philox key of the subspace core solver's starting block (stream = update: 0 row, 1 column)
constexpr uint32_t kSubSeed = 0x5eed5eedu;

int launch_status() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("HIP launch error: ") + hipGetErrorString(e));
        return FASTPI_EHIP;
    }
    return FASTPI_OK;
}

template <typename T>
int upload(std::vector<void*>& allocs, T*& dst, const T* src, size_t count, hipStream_t st) {
    dst = nullptr;
    if (count == 0) return FASTPI_OK;
    void* p = nullptr;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
        set_error("device allocation failed for a plan table");
        return FASTPI_ENOMEM;
    }
    allocs.push_back(p);
    dst = static_cast<T*>(p);
    HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, st));
    return FASTPI_OK;
}

template <typename T>
int ensure(T*& buf, size_t& have, size_t bytes, size_t cap, hipStream_t st) {
    if (bytes <= have) return FASTPI_OK;
    if (cap && bytes > cap) {
        set_error("workspace of " + std::to_string(bytes) + " bytes exceeds the cap");
        return FASTPI_ENOMEM;
    }
    if (buf) {
        hipStreamSynchronize(st);
        hipFree(buf);
        buf = nullptr;
        have = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        set_error("device workspace allocation of " + std::to_string(bytes) + " bytes failed");
        return FASTPI_ENOMEM;
    }
    buf = static_cast<T*>(p);
    have = bytes;
    return FASTPI_OK;
}

// the smallest partial-Gram height any schedule may pick (largest eigensolver workspace)
constexpr int kMinGramRows = 64;

}  // namespace

int upload_segments(std::vector<void*>& allocs, const Segments& s, SegDev& d, hipStream_t st) {
    int rc;
    d = SegDev{};
    int32_t *owner = nullptr, *pidx = nullptr, *mo = nullptr, *mp = nullptr;
    int64_t *b = nullptr, *e = nullptr;
    if ((rc = upload(allocs, owner, s.owner.data(), s.owner.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(allocs, pidx, s.pidx.data(), s.pidx.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(allocs, b, s.begin.data(), s.begin.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(allocs, e, s.end.data(), s.end.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(allocs, mo, s.multi_owner.data(), s.multi_owner.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(allocs, mp, s.multi_ptr.data(), s.multi_ptr.size(), st)) != FASTPI_OK) return rc;
    d.owner = owner;
    d.pidx = pidx;
    d.begin = b;
    d.end = e;
    d.multi_owner = mo;
    d.multi_ptr = mp;
    d.nseg = static_cast<int64_t>(s.owner.size());
    d.nmulti = static_cast<int64_t>(s.multi_owner.size());
    d.npart = s.npart;
    return FASTPI_OK;
}

bool tuning_valid(const Tuning& t) {
    return t.block_lds >= 4096 && t.block_lds <= 60 * 1024 && t.block_wgs_per_cu >= 1 &&
           t.block_wgs_per_cu <= 16 && eig_gram_rows_valid(t.gram_rows) &&
           (t.inner_sweeps == 1 || t.inner_sweeps == 2) && (t.precond == 0 || t.precond == 1) &&
           t.core_mode >= -1 && t.core_mode <= 1 && (t.eig_fused == 0 || t.eig_fused == 1);
}

bool inner_valid(const InnerCfg& c) {
    return c.mode >= 0 && c.mode <= 2 && c.oversample >= 0 && c.oversample <= 256 && c.iters >= 0 && c.iters <= 64;
}

bool inner_applies(const InnerCfg& c, int64_t t, int64_t q) {
    if (c.mode == 0 || t <= 0 || t + c.oversample >= q) return false;
    return c.mode == 2 || t < static_cast<int64_t>(std::ceil(0.3 * static_cast<double>(q)));
}

bool core_cfg_valid(const CoreCfg& c) {
    return (c.mode == 0 || c.mode == 1) && c.min_order >= 64 && c.k_factor >= 1.0 && c.k_factor <= 8.0 &&
           c.k_factor_mixed >= 1.0 && c.k_factor_mixed <= 8.0 &&
           c.max_frac > 0.0 && c.max_frac <= 1.0 && c.iters_fp64 >= 1 && c.iters_fp64 <= 256 &&
           c.iters_mixed >= 1 && c.iters_mixed <= 256 && c.orth_every >= 1 && c.orth_every <= 4 &&
           c.res_tol_fp64 > 0 && c.res_tol_mixed > 0;
}

int64_t core_basis(const CoreCfg& c, int64_t t, int64_t q, bool mixed) {
    if (c.mode == 0 || q < c.min_order || t <= 0) return 0;
    const double f = mixed ? c.k_factor_mixed : c.k_factor;
    const int64_t k = (static_cast<int64_t>(std::ceil(f * static_cast<double>(t))) + 31) / 32 * 32;
    if (k <= t || static_cast<double>(k) > c.max_frac * static_cast<double>(q)) return 0;
    return k;
}

void instance_free(Instance& I, hipStream_t st) {
    if (!I.allocs.empty() || I.ws || I.iws) hipStreamSynchronize(st);
    for (void* p : I.allocs) hipFree(p);
    if (I.ws) hipFree(I.ws);
    if (I.iws) hipFree(I.iws);
    int* status = I.status;
    I = Instance{};
    I.status = status;
}

int instance_upload(Instance& I, const Plan& p, size_t ws_cap, hipStream_t st) {
    if (!I.allocs.empty()) hipStreamSynchronize(st);
    for (void* a : I.allocs) hipFree(a);
    I.allocs.clear();
    I.dp = DevicePlan{};
    DevicePlan& d = I.dp;
    d.m = p.m;
    d.n = p.n;
    d.nnz = p.nnz;
    d.m1 = p.ro.m1;
    d.n1 = p.ro.n1;
    d.m2 = p.ro.m2;
    d.n2 = p.ro.n2;
    d.s_b = p.s_b;
    d.s = p.s;
    d.r = p.r;
    d.B_dense = p.B_dense;
    d.val_elems = p.val_elems;
    d.blk_elems = p.blk_elems;
    d.u1 = p.u1_elems;
    d.v1 = p.v1_elems;
    d.off_a21r = p.off_a21r;
    d.off_a21c = p.off_a21c;
    d.off_tr = p.off_tr;
    d.off_tc = p.off_tc;
    // Every block gets global scratch for its X and J, so any LDS budget of the persistent
    // launch can fall back to it.
    I.work = p.work;
    I.scratch_off.assign(p.work.size(), 0);
    int64_t gs = 0;
    for (size_t i = 0; i < p.work.size(); ++i) {
        const BlockWork& w = p.work[i];
        const int64_t pp = std::max(w.rows, w.cols), qq = std::min(w.rows, w.cols);
        I.scratch_off[i] = gs;
        // X and J (in FP64 size, enough for either compute type), then for more than 256
        // columns their norms (q doubles) and ranks (q ints)
        const int64_t extra = qq > 256 ? 2 * qq : 0;
        gs += ((pp * qq + qq * qq + extra + 31) / 32) * 32;
    }
    int rc;
    if ((rc = upload(I.allocs, d.work, p.work.data(), p.work.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.dst0, p.dst0.data(), p.dst0.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.dst1, p.dst1.data(), p.dst1.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.a21_rowptr, p.a21_rowptr.data(), p.a21_rowptr.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.a21_colptr, p.a21_colptr.data(), p.a21_colptr.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.t_rowptr, p.t_rowptr.data(), p.t_rowptr.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.t_colptr, p.t_colptr.data(), p.t_colptr.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.a21_colidx, p.a21_colidx.data(), p.a21_colidx.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.a21_rowidx, p.a21_rowidx.data(), p.a21_rowidx.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.t_colidx, p.t_colidx.data(), p.t_colidx.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.t_rowidx, p.t_rowidx.data(), p.t_rowidx.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.piT, p.ro.piT.data(), p.ro.piT.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.invF, p.invF.data(), p.invF.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload(I.allocs, d.invT, p.invT.data(), p.invT.size(), st)) != FASTPI_OK) return rc;
    if ((rc = upload_segments(I.allocs, p.seg_a21c, d.seg_a21c, st)) != FASTPI_OK) return rc;
    if ((rc = upload_segments(I.allocs, p.seg_a21r, d.seg_a21r, st)) != FASTPI_OK) return rc;
    if ((rc = upload_segments(I.allocs, p.seg_tc, d.seg_tc, st)) != FASTPI_OK) return rc;
    if ((rc = upload_segments(I.allocs, p.seg_tr, d.seg_tr, st)) != FASTPI_OK) return rc;

    // workspace layout (doubles)
    const int64_t m = d.m, n1 = d.n1, n2 = d.n2, s = d.s, r = d.r;
    const int64_t q3 = s + n2;
    int64_t o = 0;
    auto take = [&o](int64_t cnt) {
        const int64_t at = o;
        o += ((cnt + 31) / 32) * 32;
        return at;
    };
    I.o_vals = take(d.val_elems);
    I.o_u1 = take(d.u1);
    I.o_v1 = take(d.v1);
    I.o_sig1 = take(d.s_b);
    I.o_g2 = take(n1 * n1);
    I.o_v2 = take(n1 * s);
    I.o_lam2 = take(s);
    I.o_sig2 = take(s);
    I.o_inv2 = take(s);
    I.o_u2 = take(m * s);
    I.o_g3 = take(q3 * q3);
    I.o_vt = take(q3 * r);
    I.o_lam3 = take(r);
    I.o_sig3 = take(r);
    I.o_inv3 = take(r);
    I.o_c1 = take(s * r);
    I.o_c2 = take(n2 * r);
    I.o_eig = take(static_cast<int64_t>(std::max(eig_job_doubles(std::max<int64_t>(n1, 1), kMinGramRows),
                                                 eig_job_doubles(std::max<int64_t>(q3, 1), kMinGramRows))));
    const int sp = std::max(gemm_tn_splits(s, s, m, false), gemm_tn_splits(s, s, m, true));   // either form
    I.o_part = take(static_cast<int64_t>(sp) * s * s);
    I.o_gs = take(gs);
    const int64_t spart = std::max({p.seg_a21c.npart * n1, p.seg_tc.npart * std::max(n2, s),
                                    p.seg_a21r.npart * s, p.seg_tr.npart * r, int64_t(1)});
    I.o_spart = take(spart);
    I.o_end = o;
    if ((rc = ensure(I.ws, I.ws_bytes, static_cast<size_t>(o) * sizeof(double), ws_cap, st)) != FASTPI_OK)
        return rc;
    const size_t ints = std::max(eig_job_ints(std::max<int64_t>(n1, 1)), eig_job_ints(std::max<int64_t>(q3, 1)));
    if ((rc = ensure(I.iws, I.iws_bytes, ints * sizeof(int), 0, st)) != FASTPI_OK) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    d.valid = true;
    return launch_status();
}

// ---------------------------------------------------------------------------------------
// group
// ---------------------------------------------------------------------------------------
static void free_rand(Group& g);
static void free_sub(Group& g);

void group_drop_graphs(Group& g) {
    for (hipGraphExec_t* e : {&g.g_front, &g.g_sw1, &g.g_front2, &g.g_sw2, &g.g_mid, &g.g_sw3, &g.g_back}) {
        if (*e) hipGraphExecDestroy(*e);
        *e = nullptr;
    }
    g.key.clear();
}

void group_free(Group& g) {
    group_drop_graphs(g);
    if (g.tasks) hipFree(g.tasks);
    if (g.counter) hipFree(g.counter);
    g.tasks = nullptr;
    g.counter = nullptr;
    g.ntasks = 0;
    eig_set_free(g.set1);
    eig_set_free(g.set2);
    eig_set_free(g.set3);
    free_rand(g);
    free_sub(g);
    for (void* p : g.ballocs) hipFree(p);
    g.ballocs.clear();
    if (g.cap) hipStreamDestroy(g.cap);
    g.cap = nullptr;
}

static void free_sub(Group& g) {
    for (int c = 0; c < 2; ++c) {
        SubSet& S = g.sub[c];
        eig_set_free(S.fb);
        if (S.dchol) hipFree(S.dchol);
        if (S.flags) hipFree(S.flags);
        if (S.host_flags) hipHostFree(S.host_flags);
        for (void* p : S.allocs) hipFree(p);
        S = SubSet{};
    }
}

// C (q x n) = G B for a core on the subspace route, through the core's K split and partials
// when it has one (n <= k, so the partials fit); timed under `kind` when a timer is given.
static void product_by_g(const SubCore& R, const double* B, int64_t n, double* C, bool fp32, hipStream_t st,
                         KernelTimer* timer = nullptr, int kind = KT_NONE) {
    if (R.gsplit > 1) {
        launch_mfma_gemm(false, false, R.G, R.q, B, n, R.q, n, R.q, R.gpart, n, R.gsplit, R.q * n, st, fp32, timer,
                         kind);
        launch_sum_parts(R.gpart, R.gsplit, R.q, n, C, n, st);
    } else {
        launch_gemm_nn(R.G, R.q, nullptr, B, n, R.q, n, R.q, C, n, nullptr, st, fp32, timer, kind);
    }
}

// Buffers of one core on the subspace route and its Rayleigh-Ritz eigensolver job.
static int make_sub_core(Group& g, SubSet& S, int inst, int64_t q, int64_t t, int64_t k, const double* G,
                         double* lam_out, double* vec_out, EigJob& hjob, hipStream_t st) {
    const Instance& I = *g.inst[inst];
    SubCore R;
    R.inst = inst;
    R.q = q;
    R.t = t;
    R.k = k;
    R.kp = static_cast<int>((k + 63) / 64 * 64);
    R.G = G;
    R.lam_out = lam_out;
    R.vec_out = vec_out;
    R.sp = gemm_tn_splits(k, k, q, false, g.ncu);
    // the q x k products by G (128 x 128 tiles) split K so that their workgroups fill whole
    // waves of the resident slots: two workgroups per compute unit for the FP32 kernel of the
    // mixed form, one for the FP64 kernel. The split s minimises ceil(tiles s / slots) / s (the
    // product's time in units of one unsplit wave) plus 0.02 s for the partials written and
    // summed, with chunks of at least 256 rows of K
    const int64_t tiles = ((q + 127) / 128) * ((k + 127) / 128);
    const int64_t slots = static_cast<int64_t>(g.mixed ? 2 : 1) * g.ncu;
    const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(16, q / 256));
    R.gsplit = 1;
    double best = 1e30;
    for (int64_t s = 1; s <= smax; ++s) {
        const double c = static_cast<double>((tiles * s + slots - 1) / slots) / static_cast<double>(s) + 0.02 * s;
        if (c < best - 1e-12) {
            best = c;
            R.gsplit = static_cast<int>(s);
        }
    }
    const int64_t kp = R.kp;
    const size_t ed = eig_job_doubles(k, g.tune.gram_rows), ei = eig_job_ints(k);
    const size_t doubles = static_cast<size_t>(2 * q * k + k * k + k * t + static_cast<int64_t>(R.sp) * k * k +
                                               2 * kp * kp + kp +
                                               (R.gsplit > 1 ? static_cast<int64_t>(R.gsplit) * q * k : 0)) +
                           ed;
    void* p = nullptr;
    if (hipMalloc(&p, doubles * sizeof(double) + ei * sizeof(int)) != hipSuccess) {
        set_error("device allocation failed (subspace core solver)");
        return FASTPI_ENOMEM;
    }
    S.allocs.push_back(p);
    double* b = static_cast<double*>(p);
    R.Q = b;
    R.Y = R.Q + q * k;
    R.H = R.Y + q * k;
    R.Wv = R.H + k * k;
    R.part = R.Wv + k * t;
    CholJob J{};
    J.B = R.part + static_cast<int64_t>(R.sp) * k * k;
    J.M = J.B + kp * kp;
    J.dg = J.M + kp * kp;
    R.gpart = R.gsplit > 1 ? J.dg + kp : nullptr;
    double* eigws = J.dg + kp + (R.gsplit > 1 ? static_cast<int64_t>(R.gsplit) * q * k : 0);
    int* eigiws = reinterpret_cast<int*>(eigws + ed);
    J.k = static_cast<int>(k);
    J.kp = R.kp;
    // B and M start as zeros and B holds the identity past k (neither is rewritten there)
    HIP_TRY(hipMemsetAsync(J.B, 0, sizeof(double) * static_cast<size_t>(2 * kp * kp), st));
    launch_fill_diag(J.B, kp, k, kp, 1.0, st);
    S.cores.push_back(R);
    S.chol.push_back(J);
    S.max_kp = std::max(S.max_kp, R.kp);
    // the projected matrix H starts the Jacobi as it is, without the pivoted-Cholesky start (no
    // scratch given): a Gram of a converged basis needs no fewer sweeps from that start. Its
    // cosine threshold in the mixed form (unless one is set): far below what the form's
    // residual check and gates resolve, with the eigenvalue error quadratic in it
    const double tol = g.eig_tol > 0 ? g.eig_tol : (g.mixed ? g.core.rr_tol_mixed : 0.0);
    hjob = eig_make_job(R.H, nullptr, k, t, lam_out, R.Wv, eigws, eigiws, I.status, tol, g.tune.gram_rows, inst);
    return launch_status();
}

static int finish_sub_set(Group& g, SubSet& S, std::vector<EigJob>& fbjobs, hipStream_t st) {
    const int nc = static_cast<int>(S.cores.size());
    if (nc == 0) return FASTPI_OK;
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(int) * (nc + 16)) != hipSuccess) return FASTPI_ENOMEM;
    S.flags = static_cast<int*>(p);
    if (hipHostMalloc(&p, sizeof(int) * (nc + 16), hipHostMallocDefault) != hipSuccess) return FASTPI_ENOMEM;
    S.host_flags = static_cast<int*>(p);
    for (int i = 0; i < nc; ++i) S.chol[i].flag = S.flags + i;
    if (hipMalloc(&p, sizeof(CholJob) * nc) != hipSuccess) return FASTPI_ENOMEM;
    S.dchol = static_cast<CholJob*>(p);
    HIP_TRY(hipMemcpyAsync(S.dchol, S.chol.data(), sizeof(CholJob) * nc, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    // the fallback follows the schedule like the Jacobi cores
    return eig_set_create(S.fb, fbjobs, g.tune.gram_rows, g.tune.precond != 0, g.tune.eig_fused != 0, st);
}

static void free_rand(Group& g) {
    for (int c = 0; c < 2; ++c) {
        eig_set_free(g.rset[c]);
        g.rcores[c].clear();
    }
    for (void* p : g.rallocs) hipFree(p);
    g.rallocs.clear();
}

// Buffers and eigensolver job of one randomized core (all in one allocation).
static int make_rand_core(Group& g, int inst, int64_t q, int64_t t, const double* G, double* lam_out,
                          double* vec_out, RandCore& R, EigJob& job) {
    const Instance& I = *g.inst[inst];
    R = RandCore{};
    R.inst = inst;
    R.q = q;
    R.t = t;
    R.k = t + g.inner.oversample;
    R.G = G;
    R.lam_out = lam_out;
    R.vec_out = vec_out;
    const int64_t k = R.k;
    R.sp = gemm_tn_splits(k, k, q, false, g.ncu);
    const size_t ed = eig_job_doubles(k, g.tune.gram_rows), ei = eig_job_ints(k);
    const size_t doubles = static_cast<size_t>(2 * q * k + 3 * k * k + k + static_cast<int64_t>(R.sp) * k * k) + ed;
    void* p = nullptr;
    if (hipMalloc(&p, doubles * sizeof(double) + ei * sizeof(int)) != hipSuccess) {
        set_error("device allocation failed (randomized inner solver)");
        return FASTPI_ENOMEM;
    }
    g.rallocs.push_back(p);
    double* b = static_cast<double*>(p);
    R.Y = b;
    R.Q = R.Y + q * k;
    R.W = R.Q + q * k;
    R.Wv = R.W + k * k;
    R.Ws = R.Wv + k * k;
    R.Wd = R.Ws + k * k;
    R.part = R.Wd + k;
    double* eigws = R.part + static_cast<int64_t>(R.sp) * k * k;
    int* eigiws = reinterpret_cast<int*>(eigws + ed);
    // the k x k input (a basis' Gram matrix, then the projected core) may be overwritten
    job = eig_make_job(R.W, R.W, k, k, R.Wd, R.Wv, eigws, eigiws, I.status, g.eig_tol, g.tune.gram_rows, inst);
    return FASTPI_OK;
}

static int build_sets(Group& g, hipStream_t st) {
    free_rand(g);
    free_sub(g);
    std::vector<EigJob> fj[2];
    eig_set_free(g.set1);
    for (void* p : g.ballocs) hipFree(p);
    g.ballocs.clear();
    g.sign_v2.assign(g.inst.size(), 0);
    std::vector<EigJob> j1, j2, j3, jr[2];
    int rc = FASTPI_OK;
    // blocks on the Gram route: G, E, lam, W, split-K partials and eigensolver workspace
    for (BigBlock& b : g.big) {
        const int64_t p = b.p, q = b.q, t = b.t;
        const int spg = b.trans ? gemm_tn_splits(q, q, p, false, g.ncu) : 1;
        const int spw = b.trans ? 1 : gemm_tn_splits(p, t, q, false, g.ncu);
        b.sp = std::max(spg, spw);
        // the untransposed Gram of a narrow block runs one tile over a long K: chunks of 64
        // rows on as many workgroups, their partials summed in order
        b.sp_nt = (!b.trans && q <= 256) ? static_cast<int>(std::min<int64_t>(16, std::max<int64_t>(1, p / 64))) : 1;
        const int64_t part = std::max({static_cast<int64_t>(spg) * q * q, static_cast<int64_t>(spw) * p * t,
                                       static_cast<int64_t>(b.sp_nt) * q * q});
        const size_t ed = eig_job_doubles(q, g.tune.gram_rows), ei = eig_job_ints(q);
        const size_t doubles = static_cast<size_t>(q * q + q * t + t + p * t + part) + ed;
        void* mem = nullptr;
        if (hipMalloc(&mem, doubles * sizeof(double) + ei * sizeof(int)) != hipSuccess) {
            set_error("device allocation failed (large diagonal blocks)");
            return FASTPI_ENOMEM;
        }
        g.ballocs.push_back(mem);
        b.G = static_cast<double*>(mem);
        b.E = b.G + q * q;
        b.lam = b.E + q * t;
        b.W = b.lam + t;
        b.part = b.W + p * t;
        double* ews = b.part + part;
        int* eiws = reinterpret_cast<int*>(ews + ed);
        // the status words of the block's matrix take its eigensolver's flags
        j1.push_back(eig_make_job(b.G, b.G, q, t, b.lam, b.E, ews, eiws, g.inst[b.inst]->status, g.eig_tol,
                                  g.tune.gram_rows, b.inst));
    }
    for (size_t i = 0; i < g.inst.size() && rc == FASTPI_OK; ++i) {
        Instance& I = *g.inst[i];
        const DevicePlan& d = I.dp;
        double* ws = I.ws;
        const int64_t q3 = d.s + d.n2;
        const int tag = static_cast<int>(i);
        if (d.n1 > 0 && d.s > 0) {
            if (inner_applies(g.inner, d.s, d.n1)) {
                RandCore R;
                EigJob J;
                rc = make_rand_core(g, tag, d.n1, d.s, ws + I.o_g2, ws + I.o_lam2, ws + I.o_v2, R, J);
                g.rcores[0].push_back(R);
                jr[0].push_back(J);
            } else {
                const EigJob J = eig_make_job(ws + I.o_g2, ws + I.o_g2, d.n1, d.s, ws + I.o_lam2, ws + I.o_v2,
                                              ws + I.o_eig, I.iws, I.status, g.eig_tol, g.tune.gram_rows, tag);
                const int64_t k = core_basis(g.core, d.s, d.n1, g.mixed);
                if (k > 0) {
                    EigJob H;
                    rc = make_sub_core(g, g.sub[0], tag, d.n1, d.s, k, ws + I.o_g2, ws + I.o_lam2, ws + I.o_v2, H, st);
                    j2.push_back(H);
                    fj[0].push_back(J);
                } else {
                    j2.push_back(J);
                }
            }
        }
        if (rc == FASTPI_OK && q3 > 0 && d.r > 0) {
            if (inner_applies(g.inner, d.r, q3)) {
                RandCore R;
                EigJob J;
                rc = make_rand_core(g, tag, q3, d.r, ws + I.o_g3, ws + I.o_lam3, ws + I.o_vt, R, J);
                g.rcores[1].push_back(R);
                jr[1].push_back(J);
                // its test matrix meets the columns of U2 Sigma2: fix their signs first
                g.sign_v2[i] = 1;
            } else {
                const EigJob J = eig_make_job(ws + I.o_g3, ws + I.o_g3, q3, d.r, ws + I.o_lam3, ws + I.o_vt,
                                              ws + I.o_eig, I.iws, I.status, g.eig_tol, g.tune.gram_rows, tag);
                const int64_t k = core_basis(g.core, d.r, q3, g.mixed);
                if (k > 0) {
                    EigJob H;
                    rc = make_sub_core(g, g.sub[1], tag, q3, d.r, k, ws + I.o_g3, ws + I.o_lam3, ws + I.o_vt, H, st);
                    j3.push_back(H);
                    fj[1].push_back(J);
                } else {
                    j3.push_back(J);
                }
            }
        }
    }
    if (rc != FASTPI_OK) return rc;
    // the cores are rebuilt by every run, so the factorisation may overwrite them
    // the Gram route of large blocks takes sigma = sqrt(lambda) down to 1e-7 of the largest and
    // divides by it, so its eigensolves start from the pivoted-Cholesky factor (relative
    // accuracy) whatever the schedule
    rc = eig_set_create(g.set1, j1, g.tune.gram_rows, true, g.tune.eig_fused != 0, st);
    if (rc == FASTPI_OK)
        rc = eig_set_create(g.set2, j2, g.tune.gram_rows, g.tune.precond != 0, g.tune.eig_fused != 0, st);
    if (rc == FASTPI_OK)
        rc = eig_set_create(g.set3, j3, g.tune.gram_rows, g.tune.precond != 0, g.tune.eig_fused != 0, st);
    // the randomized solver's basis Grams are numerically rank-deficient and its
    // orthonormalization divides by the square roots of their eigenvalues down to k eps of the
    // largest: those need relative accuracy, which the pivoted-Cholesky start gives (from G
    // itself they carry absolute errors of ~ld eps of the largest), whatever the schedule
    for (int c = 0; c < 2 && rc == FASTPI_OK; ++c)
        rc = eig_set_create(g.rset[c], jr[c], g.tune.gram_rows, true, g.tune.eig_fused != 0, st);
    for (int c = 0; c < 2 && rc == FASTPI_OK; ++c) rc = finish_sub_set(g, g.sub[c], fj[c], st);
    if (rc != FASTPI_OK) set_error("eigensolver set allocation failed");
    return rc;
}

// Subspace core solver for the cores of update c (0: row, 1: column) on that route: start
// from a Gaussian block Q (k columns), then `iters` products Y = G Q, the block orthonormalised
// (Cholesky QR: Y^T Y = L L^T, Q = Y L^-T) before every orth_every-th product; in the mixed
// form the products by G and by L^-T run in FP32 (the Gram and the factorisation in FP64). Then two FP64 orthonormalisations,
// H = Q^T G Q, its top t eigenpairs (W, lambda) by the block Jacobi eigensolver, vectors Q W.
// Every core's result is checked (the residual of each pair, the rank of every Cholesky QR);
// the host reads the checks and solves the failing set again with Jacobi on G.
static void sub_pre(Group& g, int c, const RunCfg& cfg, KernelTimer* timer, hipStream_t st) {
    SubSet& S = g.sub[c];
    if (S.cores.empty()) return;
    const bool mixed = cfg.mixed;
    const int iters = mixed ? g.core.iters_mixed : g.core.iters_fp64;
    const int nc = static_cast<int>(S.cores.size());
    launch_fill_i32(S.flags, nc, 0, st);
    for (SubCore& R : S.cores) launch_gauss(R.Q, R.q * R.k, kSubSeed, static_cast<uint32_t>(c), st);
    bool in_q = true;
    auto cur = [&](SubCore& R) { return in_q ? R.Q : R.Y; };
    auto oth = [&](SubCore& R) { return in_q ? R.Y : R.Q; };
    // the block's Gram matrix is always formed in FP64: an FP32 Gram of a block whose
    // condition grew over two products can lose definiteness
    auto orth = [&](bool fp32) {
        for (int i = 0; i < nc; ++i) {
            SubCore& R = S.cores[i];
            launch_gemm_tn(cur(R), R.k, cur(R), R.k, R.k, R.k, R.q, S.chol[i].B, R.kp, nullptr, nullptr, R.part, R.sp,
                           st, false);
        }
        launch_chol_inverse(S.dchol, nc, S.max_kp, st, timer);
        for (int i = 0; i < nc; ++i) {
            SubCore& R = S.cores[i];
            launch_gemm_nt(cur(R), R.k, S.chol[i].M, R.kp, R.q, R.k, R.k, oth(R), R.k, st, fp32, nullptr);
        }
        in_q = !in_q;
    };
    auto apply = [&](bool fp32) {
        for (SubCore& R : S.cores) product_by_g(R, cur(R), R.k, oth(R), fp32, st, timer, KT_SUB_GEMM);
        in_q = !in_q;
    };
    for (int it = 0; it < iters; ++it) {
        if (it % g.core.orth_every == 0) orth(mixed);
        apply(mixed);
    }
    orth(false);
    orth(false);
    // H = Q^T (G Q), a job of the update's batched Jacobi set
    for (SubCore& R : S.cores) {
        product_by_g(R, cur(R), R.k, oth(R), false, st);
        launch_gemm_tn(cur(R), R.k, oth(R), R.k, R.k, R.k, R.q, R.H, R.k, nullptr, nullptr, R.part, R.sp, st, false);
        launch_symmetrize(R.H, R.k, st);
    }
    S.basis_in_q = in_q;
}

static int sub_post(Group& g, int c, const RunCfg& cfg, hipStream_t st) {
    SubSet& S = g.sub[c];
    S.fallbacks = 0;
    if (S.cores.empty()) return FASTPI_OK;
    const double tol = cfg.mixed ? g.core.res_tol_mixed : g.core.res_tol_fp64;
    const int nc = static_cast<int>(S.cores.size());
    const bool in_q = S.basis_in_q;
    for (int i = 0; i < nc; ++i) {
        SubCore& R = S.cores[i];
        const double* Qb = in_q ? R.Q : R.Y;
        double* Rb = in_q ? R.Y : R.Q;
        launch_gemm_nn(Qb, R.k, nullptr, R.Wv, R.t, R.q, R.t, R.k, R.vec_out, R.t, nullptr, st, false);
        product_by_g(R, R.vec_out, R.t, Rb, false, st);
        launch_sub_residual(Rb, R.vec_out, R.lam_out, R.q, R.t, tol, S.flags + i, st);
    }
    HIP_TRY(hipMemcpyAsync(S.host_flags, S.flags, sizeof(int) * nc, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < nc; ++i) S.fallbacks += S.host_flags[i] != 0 ? 1 : 0;
    if (S.fallbacks > 0) {
        eig_begin(S.fb, st);
        const int rc = eig_iterate(S.fb, cfg.max_sweeps, g.tune.inner_sweeps, st, cfg.copy_st, cfg.timer, nullptr);
        if (rc != FASTPI_OK) return rc;
        eig_end(S.fb, st);
    }
    return launch_status();
}

int group_set_core(Group& g, const CoreCfg& c, hipStream_t st) {
    if (!core_cfg_valid(c)) {
        set_error("invalid core-solver parameters");
        return FASTPI_EINVAL;
    }
    g.core = c;
    group_drop_graphs(g);
    if (!g.inst.empty() && g.counter) {
        HIP_TRY(hipStreamSynchronize(st));
        return build_sets(g, st);
    }
    return FASTPI_OK;
}

// Randomized subspace iteration for the cores of update c (0: row, 1: column): Y = G Omega;
// `iters` products by G, orthonormalized before every other one; two final
// orthonormalizations; the Rayleigh-Ritz eigenpairs of B^T G B give the top t pairs (vectors
// B W_t). orth(Y) = Y V diag(d^-1/2) for
// the eigenpairs (d, V) of Y^T Y, which spans the same subspace as any other orthonormalization.
static int rand_run(Group& g, int c, const RunCfg& cfg, hipStream_t st) {
    std::vector<RandCore>& cores = g.rcores[c];
    if (cores.empty()) return FASTPI_OK;
    EigSet& es = g.rset[c];
    for (RandCore& R : cores) {
        R.sweeps = 0;
        R.rotated = 0;
    }
    auto eig = [&]() -> int {
        eig_begin(es, st);
        const int rc = eig_iterate(es, cfg.max_sweeps, g.tune.inner_sweeps, st, cfg.copy_st, cfg.timer, nullptr);
        if (rc != FASTPI_OK) return rc;
        eig_end(es, st);
        for (int j = 0; j < es.njobs; ++j)
            for (RandCore& R : cores)
                if (R.inst == es.host[j].tag) {
                    R.sweeps += es.host_state[kEigStateWords * j + kEigStSweeps];
                    R.rotated += es.host_state[kEigStateWords * j + kEigStTotal];
                }
        return FASTPI_OK;
    };
    // src -> dst: dst = src V diag(d^-1/2) over the eigenpairs of src^T src
    auto orth = [&](bool from_y) -> int {
        for (RandCore& R : cores) {
            const double* src = from_y ? R.Y : R.Q;
            launch_gemm_tn(src, R.k, src, R.k, R.k, R.k, R.q, R.W, R.k, nullptr, nullptr, R.part, R.sp, st, false);
        }
        const int rc = eig();
        if (rc != FASTPI_OK) return rc;
        for (RandCore& R : cores) {
            launch_scale_cols(R.Wv, R.Wd, R.k, static_cast<double>(R.k) * DBL_EPSILON, R.Ws, st);
            launch_gemm_nn(from_y ? R.Y : R.Q, R.k, nullptr, R.Ws, R.k, R.q, R.k, R.k, from_y ? R.Q : R.Y, R.k,
                           nullptr, st, false);
        }
        return FASTPI_OK;
    };
    for (RandCore& R : cores) {
        launch_gauss(R.Q, R.q * R.k, g.inner.seed, static_cast<uint32_t>(c), st);
        launch_gemm_nn(R.G, R.q, nullptr, R.Q, R.k, R.q, R.k, R.q, R.Y, R.k, nullptr, st, false);
    }
    int rc;
    // the current block alternates between Y and Q; every other power iteration skips the
    // orthonormalization (the subspace is the same in exact arithmetic, and one product by G
    // squares the block's condition number at most once between two of them)
    bool in_y = true;
    auto apply = [&]() {
        for (RandCore& R : cores)
            launch_gemm_nn(R.G, R.q, nullptr, in_y ? R.Y : R.Q, R.k, R.q, R.k, R.q, in_y ? R.Q : R.Y, R.k,
                           nullptr, st, false);
        in_y = !in_y;
    };
    auto normalize = [&]() -> int {
        const int r = orth(in_y);
        in_y = !in_y;
        return r;
    };
    for (int it = 0; it < g.inner.iters; ++it) {
        if (it % 2 == 0 && (rc = normalize()) != FASTPI_OK) return rc;
        apply();
    }
    if ((rc = normalize()) != FASTPI_OK) return rc;
    if ((rc = normalize()) != FASTPI_OK) return rc;   // re-orthonormalized basis B
    // Rayleigh-Ritz: H = B^T (G B), its eigenpairs, vectors B W_t
    for (RandCore& R : cores) {
        const double* B = in_y ? R.Y : R.Q;
        double* GB = in_y ? R.Q : R.Y;
        launch_gemm_nn(R.G, R.q, nullptr, B, R.k, R.q, R.k, R.q, GB, R.k, nullptr, st, false);
        launch_gemm_tn(B, R.k, GB, R.k, R.k, R.k, R.q, R.W, R.k, nullptr, nullptr, R.part, R.sp, st, false);
    }
    if ((rc = eig()) != FASTPI_OK) return rc;
    for (RandCore& R : cores) {
        launch_gemm_nn(in_y ? R.Y : R.Q, R.k, nullptr, R.Wv, R.k, R.q, R.t, R.k, R.vec_out, R.t, nullptr, st, false);
        launch_copy(R.Wd, R.t, R.lam_out, st);
    }
    return launch_status();
}

int group_build(Group& g, int device, hipStream_t st) {
    Group fresh;
    fresh.inst = g.inst;
    fresh.tune = g.tune;
    fresh.inner = g.inner;
    fresh.core = g.core;
    fresh.big_cost = g.big_cost;
    fresh.eig_tol = g.eig_tol;
    group_free(g);
    g = fresh;
    HIP_TRY(hipDeviceGetAttribute(&g.ncu, hipDeviceAttributeMultiprocessorCount, device));
    if (g.ncu <= 0) g.ncu = 256;
    // all blocks of all instances, largest cost (p q^2) first
    std::vector<std::pair<double, BlockTask>> all;
    for (size_t ii = 0; ii < g.inst.size(); ++ii) {
        Instance& I = *g.inst[ii];
        if (!I.dp.valid) {
            set_error("instance without an uploaded plan");
            return FASTPI_EINVAL;
        }
        double* ws = I.ws;
        for (size_t k = 0; k < I.work.size(); ++k) {
            const BlockWork& w = I.work[k];
            BlockTask t{};
            t.A = ws + I.o_vals + w.data_off;
            t.U = ws + I.o_u1 + w.u_off;
            t.V = ws + I.o_v1 + w.v_off;
            t.sig = ws + I.o_sig1 + w.sig_off;
            t.scratch = ws + I.o_gs + I.scratch_off[k];
            t.status = I.status;
            t.rows = w.rows;
            t.cols = w.cols;
            t.rank = w.rank;
            const double pp = std::max(w.rows, w.cols), qq = std::min(w.rows, w.cols);
            if (pp * qq * qq >= g.big_cost && w.rank > 0 && qq >= 2) {
                BigBlock b;
                b.inst = static_cast<int>(ii);
                b.A = t.A;
                b.U = t.U;
                b.V = t.V;
                b.sig = t.sig;
                b.rows = w.rows;
                b.cols = w.cols;
                b.trans = w.rows < w.cols;
                b.p = static_cast<int64_t>(pp);
                b.q = static_cast<int64_t>(qq);
                b.t = w.rank;
                g.big.push_back(b);
                continue;
            }
            all.emplace_back(pp * qq * qq, t);
        }
    }
    std::stable_sort(all.begin(), all.end(),
                     [](const std::pair<double, BlockTask>& a, const std::pair<double, BlockTask>& b) {
                         return a.first > b.first;
                     });
    std::vector<BlockTask> tasks;
    tasks.reserve(all.size());
    for (auto& e : all) tasks.push_back(e.second);
    g.ntasks = static_cast<int>(tasks.size());
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(int) * 64) != hipSuccess) {
        set_error("device allocation failed (work queue)");
        return FASTPI_ENOMEM;
    }
    g.counter = static_cast<int*>(p);
    if (!tasks.empty()) {
        if (hipMalloc(&p, sizeof(BlockTask) * tasks.size()) != hipSuccess) {
            set_error("device allocation failed (block tasks)");
            return FASTPI_ENOMEM;
        }
        g.tasks = static_cast<BlockTask*>(p);
        HIP_TRY(hipMemcpyAsync(g.tasks, tasks.data(), sizeof(BlockTask) * tasks.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    int rc = build_sets(g, st);
    if (rc != FASTPI_OK) return rc;
    HIP_TRY(hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking));
    return launch_status();
}

int group_set_inner(Group& g, const InnerCfg& c, hipStream_t st) {
    if (!inner_valid(c)) {
        set_error("invalid inner-solver parameters (mode 0-2, oversample 0-256, iterations 0-64)");
        return FASTPI_EINVAL;
    }
    g.inner = c;
    group_drop_graphs(g);
    if (!g.inst.empty() && g.counter) {
        HIP_TRY(hipStreamSynchronize(st));
        return build_sets(g, st);
    }
    return FASTPI_OK;
}

int group_set_tuning(Group& g, const Tuning& t, hipStream_t st) {
    if (!tuning_valid(t)) {
        set_error("invalid schedule parameters");
        return FASTPI_EINVAL;
    }
    bool resize = t.gram_rows != g.tune.gram_rows || t.precond != g.tune.precond;
    if (t.core_mode >= 0 && t.core_mode != g.core.mode) {
        g.core.mode = t.core_mode;
        resize = true;
    }
    g.tune = t;
    group_drop_graphs(g);
    if (resize && !g.inst.empty()) {
        HIP_TRY(hipStreamSynchronize(st));
        return build_sets(g, st);
    }
    return FASTPI_OK;
}

// ---- stages ----------------------------------------------------------------------------
static void stage_front(Group& g, const double* const* val, const RunCfg& c, hipStream_t st, KernelTimer* timer) {
    for (size_t i = 0; i < g.inst.size(); ++i) {
        Instance& I = *g.inst[i];
        const DevicePlan& d = I.dp;
        double* vals = I.ws + I.o_vals;
        launch_fill_i32(I.status, 2, 0, st);
        // a1: split the reordered matrix into dense A11 blocks, A21 and T
        launch_fill(vals, d.blk_elems, 0.0, st);
        launch_gather(val[i], d.dst0, d.dst1, d.nnz, vals, I.status, st);
    }
    // a2: block SVDs (Eq. 1), every block of every instance in one persistent launch
    launch_block_svd_tasks(c.mixed, g.tasks, g.ntasks, g.counter, g.tune.block_lds, g.ncu * g.tune.block_wgs_per_cu,
                           c.max_sweeps, c.tol, st, timer);
    // large blocks: Gram matrices of their long side for the batched eigensolver
    for (BigBlock& b : g.big) {
        if (b.trans)
            launch_gemm_tn(b.A, b.q, b.A, b.q, b.q, b.q, b.p, b.G, b.q, nullptr, nullptr, b.part, b.sp, st, false);
        else if (b.sp_nt > 1) {
            launch_mfma_gemm(false, true, b.A, b.p, b.A, b.p, b.q, b.q, b.p, b.part, b.q, b.sp_nt, b.q * b.q, st,
                             false);
            launch_sum_parts(b.part, b.sp_nt, b.q, b.q, b.G, b.q, st);
        } else
            launch_gemm_nt(b.A, b.p, b.A, b.p, b.q, b.q, b.p, b.G, b.q, st, false);
    }
    eig_begin(g.set1, st);
}

static void stage_front2(Group& g, const RunCfg& c, KernelTimer* timer, hipStream_t st) {
    eig_end(g.set1, st);
    // large blocks: the other factor W = X E, then sigma and both factors into the packed
    // outputs (non-transposed: q side V, p side U; transposed: the reverse)
    for (BigBlock& b : g.big) {
        if (b.trans)
            launch_gemm_nn(b.A, b.q, nullptr, b.E, b.t, b.p, b.t, b.q, b.W, b.t, nullptr, st, false);
        else
            launch_gemm_tn(b.A, b.p, b.E, b.t, b.p, b.t, b.q, b.W, b.t, nullptr, nullptr, b.part, b.sp, st, false);
        launch_block_gram_out(b.lam, b.E, b.W, b.q, b.p, b.t, kRelCut, b.trans ? b.U : b.V, b.trans ? b.V : b.U,
                              b.sig, g.inst[b.inst]->status, st);
    }
    // a3, first half: M2^T M2 = V1 Sigma1^2 V1^T + A21^T A21
    for (Instance* Ip : g.inst) {
        Instance& I = *Ip;
        const DevicePlan& d = I.dp;
        if (!(d.n1 > 0 && d.s > 0)) continue;
        double* ws = I.ws;
        const int64_t n1 = d.n1;
        double* G2 = ws + I.o_g2;
        launch_fill(G2, n1 * n1, 0.0, st);
        launch_blockdiag_gram(d.work, static_cast<int>(d.B_dense), ws + I.o_v1, ws + I.o_sig1, G2, n1, st);
        launch_sparse_gram(d.seg_a21c, d.a21_rowidx, ws + I.o_vals + d.off_a21c, d.a21_rowptr, d.a21_colidx,
                           ws + I.o_vals + d.off_a21r, n1, G2, n1, true, ws + I.o_spart, st);
    }
    // cores on the subspace route: the iteration up to the Rayleigh-Ritz matrices, which join
    // the Jacobi set
    sub_pre(g, 0, c, timer, st);
    eig_begin(g.set2, st);
}

// after the row-update eigensolve (and eig_end of its set): the stages up to the column
// update's eigensolve
static void stage_mid(Group& g, const RunCfg& c, KernelTimer* timer, hipStream_t st) {
    for (size_t idx = 0; idx < g.inst.size(); ++idx) {
        Instance& I = *g.inst[idx];
        const DevicePlan& d = I.dp;
        double* ws = I.ws;
        double* vals = ws + I.o_vals;
        const int64_t m = d.m, m1 = d.m1, n2 = d.n2, s = d.s, r = d.r, q3 = s + n2;
        double* U2 = ws + I.o_u2;
        double* sig2 = ws + I.o_sig2;
        double* inv2 = ws + I.o_inv2;
        // a3, second half: sigma2 and U2 = M2 V2 Sigma2^-1 (block part and A21 part)
        if (d.n1 > 0 && s > 0) {
            if (idx < g.sign_v2.size() && g.sign_v2[idx]) launch_sign_fix(ws + I.o_v2, d.n1, s, st);
            launch_sqrt_inv(ws + I.o_lam2, s, kRelCut, sig2, inv2, I.status, st);
            launch_fill(U2, m * s, 0.0, st);
            launch_u2_top(d.work, static_cast<int>(d.B_dense), ws + I.o_u1, ws + I.o_sig1, ws + I.o_v1,
                          ws + I.o_v2, s, inv2, U2, I.status, st);
            launch_spmm_rows(d.seg_a21r, d.a21_colidx, vals + d.off_a21r, ws + I.o_v2, s, inv2, U2 + m1 * s, s,
                             nullptr, false, ws + I.o_spart, st);
        }
        // a4, first half: X3^T X3 for X3 = [U2 Sigma2, T]
        if (q3 > 0 && r > 0) {
            double* G3 = ws + I.o_g3;
            launch_fill(G3, q3 * q3, 0.0, st);
            if (s > 0) {
                const int sp = gemm_tn_splits(s, s, m, c.mixed, g.ncu);
                launch_gemm_tn(U2, s, U2, s, s, s, m, G3, q3, sig2, sig2, ws + I.o_part, sp, st, c.mixed);
                launch_sparse_proj(d.seg_tc, d.t_rowidx, vals + d.off_tc, U2, s, sig2, G3, q3, s, ws + I.o_spart,
                                   st);
            }
            launch_sparse_gram(d.seg_tc, d.t_rowidx, vals + d.off_tc, d.t_rowptr, d.t_colidx, vals + d.off_tr, n2,
                               G3 + s * q3 + s, q3, false, ws + I.o_spart, st);
        }
    }
    sub_pre(g, 1, c, timer, st);
    eig_begin(g.set3, st);
}

// after the column-update eigensolve (and eig_end of its set): U, S, V
static void stage_back(Group& g, double* const* U, double* const* S, double* const* V, const RunCfg& c,
                       hipStream_t st) {
    for (size_t i = 0; i < g.inst.size(); ++i) {
        Instance& I = *g.inst[i];
        const DevicePlan& d = I.dp;
        double* ws = I.ws;
        double* vals = ws + I.o_vals;
        const int64_t m = d.m, n1 = d.n1, n2 = d.n2, s = d.s, r = d.r, q3 = s + n2;
        if (!(q3 > 0 && r > 0)) continue;
        double* Vt = ws + I.o_vt;
        double* C1 = ws + I.o_c1;
        double* C2 = ws + I.o_c2;
        double* sig3 = ws + I.o_sig3;
        double* inv3 = ws + I.o_inv3;
        launch_sqrt_inv(ws + I.o_lam3, r, kRelCut, sig3, inv3, I.status, st);
        launch_col_coeffs(Vt, s, n2, r, ws + I.o_sig2, inv3, C1, C2, st);
        // a4, second half, and a5: U and V in the caller's order
        launch_gemm_nn(ws + I.o_u2, s, d.piT, C1, r, m, r, s, U[i], r, nullptr, st, c.mixed);
        launch_spmm_rows(d.seg_tr, d.t_colidx, vals + d.off_tr, C2, r, nullptr, U[i], r, d.invT, true,
                         ws + I.o_spart, st);
        launch_gemm_nn(ws + I.o_v2, s, nullptr, Vt, r, n1, r, s, V[i], r, d.invF, st, c.mixed);
        launch_copy_rows(Vt + s * r, n2, r, d.invF + n1, V[i], st);
        launch_copy(sig3, r, S[i], st);
    }
}

template <typename F>
static int capture(Group& g, F&& fn, hipGraphExec_t& out) {
    out = nullptr;
    (void)hipGetLastError();
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal));
    fn(g.cap);
    const hipError_t le = hipGetLastError();
    const hipError_t ee = hipStreamEndCapture(g.cap, &graph);
    if (le != hipSuccess || ee != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        set_error(std::string("graph capture failed: ") + hipGetErrorString(le != hipSuccess ? le : ee));
        return FASTPI_EHIP;
    }
    size_t nodes = 0;
    HIP_TRY(hipGraphGetNodes(graph, nullptr, &nodes));
    if (nodes > 0) {
        const hipError_t ie = hipGraphInstantiate(&out, graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            hipGraphDestroy(graph);
            set_error(std::string("graph instantiation failed: ") + hipGetErrorString(ie));
            return FASTPI_EHIP;
        }
    }
    hipGraphDestroy(graph);
    return FASTPI_OK;
}

static int launch_graph(Group& g, hipGraphExec_t e, hipStream_t st) {
    if (!e) return FASTPI_OK;
    ++g.graph_launches;
    HIP_TRY(hipGraphLaunch(e, st));
    return FASTPI_OK;
}

static void record_sweeps(Group& g) {
    for (Instance* I : g.inst) {
        I->sweeps[1] = I->sweeps[2] = 0;
        I->rotated[0] = I->rotated[1] = 0;
        I->route[0] = I->route[1] = 0;
    }
    // the update sets hold the Jacobi cores and the subspace cores' Rayleigh-Ritz problems (one
    // job per matrix and update either way); a fallback's Jacobi on G adds its sweeps
    const EigSet* sets[2] = {&g.set2, &g.set3};
    for (int k = 0; k < 2; ++k) {
        const EigSet& es = *sets[k];
        for (int j = 0; j < es.njobs; ++j) {
            Instance* I = g.inst[es.host[j].tag];
            I->sweeps[1 + k] = es.host_state[kEigStateWords * j + kEigStSweeps];
            I->rotated[k] = es.host_state[kEigStateWords * j + kEigStTotal];
        }
        const SubSet& S = g.sub[k];
        for (const SubCore& R : S.cores) g.inst[R.inst]->route[k] = 1;
        if (S.fallbacks > 0)
            for (int j = 0; j < S.fb.njobs; ++j) {
                Instance* I = g.inst[S.fb.host[j].tag];
                I->sweeps[1 + k] += S.fb.host_state[kEigStateWords * j + kEigStSweeps];
                I->rotated[k] += S.fb.host_state[kEigStateWords * j + kEigStTotal];
                I->route[k] = 2;
            }
        for (const RandCore& R : g.rcores[k]) {
            g.inst[R.inst]->sweeps[1 + k] = R.sweeps;
            g.inst[R.inst]->rotated[k] = R.rotated;
            g.inst[R.inst]->route[k] = 3;
        }
    }
}

int group_svd(Group& g, const double* const* val, double* const* U, double* const* S, double* const* V,
              const RunCfg& c) {
    hipStream_t st = c.st;
    int rc;
    g.graph_launches = 0;
    if (c.mixed != g.mixed) {
        // the subspace route (basis, Rayleigh-Ritz threshold) depends on the precision form:
        // rebuild the sets where a core takes it in either form
        bool differs = false;
        for (const Instance* I : g.inst) {
            const DevicePlan& d = I->dp;
            for (bool m : {false, true})
                differs = differs || core_basis(g.core, d.s, d.n1, m) > 0 || core_basis(g.core, d.r, d.s + d.n2, m) > 0;
        }
        g.mixed = c.mixed;
        if (differs && g.counter) {
            group_drop_graphs(g);
            HIP_TRY(hipStreamSynchronize(st));
            if ((rc = build_sets(g, st)) != FASTPI_OK) return rc;
        }
    }
    if (!c.use_graph) {
        stage_front(g, val, c, st, c.timer);
        if ((rc = eig_iterate(g.set1, c.max_sweeps, g.tune.inner_sweeps, st, c.copy_st, c.timer, nullptr)) !=
            FASTPI_OK)
            return rc;
        stage_front2(g, c, c.timer, st);
        if ((rc = eig_iterate(g.set2, c.max_sweeps, g.tune.inner_sweeps, st, c.copy_st, c.timer, nullptr)) !=
            FASTPI_OK)
            return rc;
        if ((rc = rand_run(g, 0, c, st)) != FASTPI_OK) return rc;
        eig_end(g.set2, st);
        if ((rc = sub_post(g, 0, c, st)) != FASTPI_OK) return rc;
        stage_mid(g, c, c.timer, st);
        if ((rc = eig_iterate(g.set3, c.max_sweeps, g.tune.inner_sweeps, st, c.copy_st, c.timer, nullptr)) !=
            FASTPI_OK)
            return rc;
        if ((rc = rand_run(g, 1, c, st)) != FASTPI_OK) return rc;
        eig_end(g.set3, st);
        if ((rc = sub_post(g, 1, c, st)) != FASTPI_OK) return rc;
        stage_back(g, U, S, V, c, st);
        record_sweeps(g);
        return launch_status();
    }
    // graphs bake in every pointer and scalar: recapture when any of them changes
    std::vector<uint64_t> key;
    for (size_t i = 0; i < g.inst.size(); ++i) {
        key.push_back(reinterpret_cast<uintptr_t>(val[i]));
        key.push_back(reinterpret_cast<uintptr_t>(U[i]));
        key.push_back(reinterpret_cast<uintptr_t>(S[i]));
        key.push_back(reinterpret_cast<uintptr_t>(V[i]));
    }
    uint64_t tol_bits = 0;
    std::memcpy(&tol_bits, &c.tol, sizeof(tol_bits));
    key.push_back(c.mixed ? 1u : 0u);
    key.push_back(static_cast<uint64_t>(c.max_sweeps));
    key.push_back(tol_bits);
    if (key != g.key || !g.g_front) {
        group_drop_graphs(g);
        HIP_TRY(hipStreamSynchronize(st));
        if ((rc = capture(g, [&](hipStream_t s) { stage_front(g, val, c, s, nullptr); }, g.g_front)) != FASTPI_OK)
            return rc;
        if (g.set1.njobs > 0 &&
            (rc = capture(g, [&](hipStream_t s) { eig_sweep(g.set1, c.max_sweeps, g.tune.inner_sweeps, s, nullptr); },
                          g.g_sw1)) != FASTPI_OK)
            return rc;
        if ((rc = capture(g, [&](hipStream_t s) { stage_front2(g, c, nullptr, s); }, g.g_front2)) != FASTPI_OK)
            return rc;
        if (g.set2.njobs > 0 &&
            (rc = capture(g, [&](hipStream_t s) { eig_sweep(g.set2, c.max_sweeps, g.tune.inner_sweeps, s, nullptr); },
                          g.g_sw2)) != FASTPI_OK)
            return rc;
        if ((rc = capture(g, [&](hipStream_t s) { stage_mid(g, c, nullptr, s); }, g.g_mid)) != FASTPI_OK) return rc;
        if (g.set3.njobs > 0 &&
            (rc = capture(g, [&](hipStream_t s) { eig_sweep(g.set3, c.max_sweeps, g.tune.inner_sweeps, s, nullptr); },
                          g.g_sw3)) != FASTPI_OK)
            return rc;
        if ((rc = capture(g, [&](hipStream_t s) { stage_back(g, U, S, V, c, s); }, g.g_back)) != FASTPI_OK)
            return rc;
        g.key = key;
    }
    if ((rc = launch_graph(g, g.g_front, st)) != FASTPI_OK) return rc;
    if ((rc = eig_iterate(g.set1, c.max_sweeps, g.tune.inner_sweeps, st, c.copy_st, nullptr, g.g_sw1)) != FASTPI_OK)
        return rc;
    if ((rc = launch_graph(g, g.g_front2, st)) != FASTPI_OK) return rc;
    if ((rc = eig_iterate(g.set2, c.max_sweeps, g.tune.inner_sweeps, st, c.copy_st, nullptr, g.g_sw2)) != FASTPI_OK)
        return rc;
    RunCfg eager = c;
    eager.timer = nullptr;
    if ((rc = rand_run(g, 0, eager, st)) != FASTPI_OK) return rc;
    eig_end(g.set2, st);
    if ((rc = sub_post(g, 0, eager, st)) != FASTPI_OK) return rc;
    if ((rc = launch_graph(g, g.g_mid, st)) != FASTPI_OK) return rc;
    if ((rc = eig_iterate(g.set3, c.max_sweeps, g.tune.inner_sweeps, st, c.copy_st, nullptr, g.g_sw3)) != FASTPI_OK)
        return rc;
    if ((rc = rand_run(g, 1, eager, st)) != FASTPI_OK) return rc;
    eig_end(g.set3, st);
    if ((rc = sub_post(g, 1, eager, st)) != FASTPI_OK) return rc;
    if ((rc = launch_graph(g, g.g_back, st)) != FASTPI_OK) return rc;
    record_sweeps(g);
    return launch_status();
}

// ---------------------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------------------
static int log2_bucket(int64_t x) {
    int b = 0;
    while (x > 1) {
        x >>= 1;
        ++b;
    }
    return b;
}

static std::string tuning_key(const Group& g, int device, bool mixed) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    std::ostringstream k;
    // the core orders from the matrices' shapes (not from the eigensolver sets, whose jobs
    // depend on the core route the schedule itself chooses)
    int64_t q2 = 0, q3 = 0;
    for (const Instance* I : g.inst) {
        q2 = std::max(q2, I->dp.n1);
        q3 = std::max(q3, I->dp.s + I->dp.n2);
    }
    k << arch << ' ' << (mixed ? "mixed" : "fp64") << " inst" << log2_bucket(static_cast<int64_t>(g.inst.size()))
      << " blk" << log2_bucket(g.ntasks) << " q2_" << log2_bucket(q2) << " q3_" << log2_bucket(q3);
    return k.str();
}

int tuning_lookup(const Group& g, const char* cache, int device, bool mixed, Tuning& out) {
    if (!cache) return 0;
    std::ifstream f(cache);
    if (!f) return 0;
    const std::string key = tuning_key(g, device, mixed);
    std::string line;
    int found = 0;
    while (std::getline(f, line)) {
        const size_t bar = line.find('|');
        if (bar == std::string::npos || line.substr(0, bar) != key) continue;
        std::istringstream v(line.substr(bar + 1));
        Tuning t;
        if (v >> t.block_lds >> t.block_wgs_per_cu >> t.gram_rows >> t.inner_sweeps >> t.precond) {
            int cm = -1, ef = 1;
            if (v >> cm) t.core_mode = cm;   // optional sixth field
            if (v >> ef) t.eig_fused = ef;   // optional seventh field
            if (!tuning_valid(t)) continue;
            out = t;
            found = 1;   // the last matching line wins
        }
    }
    return found;
}

static int store_tuning(const Group& g, const char* cache, int device, bool mixed, const Tuning& t) {
    const std::string key = tuning_key(g, device, mixed);
    std::vector<std::string> keep;
    {
        std::ifstream f(cache);
        std::string line;
        while (f && std::getline(f, line)) {
            const size_t bar = line.find('|');
            if (bar != std::string::npos && line.substr(0, bar) == key) continue;
            if (!line.empty()) keep.push_back(line);
        }
    }
    std::ofstream o(cache, std::ios::trunc);
    if (!o) {
        set_error(std::string("cannot write the tuning cache ") + cache);
        return FASTPI_EINVAL;
    }
    for (const std::string& l : keep) o << l << '\n';
    o << key << '|' << t.block_lds << ' ' << t.block_wgs_per_cu << ' ' << t.gram_rows << ' ' << t.inner_sweeps
      << ' ' << t.precond << ' ' << t.core_mode << ' ' << t.eig_fused << '\n';
    return FASTPI_OK;
}

int group_autotune(Group& g, const double* const* val, double* const* U, double* const* S, double* const* V,
                   const RunCfg& c0, const char* cache, int device, std::string* report) {
    RunCfg c = c0;
    c.use_graph = false;
    c.timer = nullptr;
    hipStream_t st = c.st;
    std::ostringstream rep;
    Tuning t;
    if (tuning_lookup(g, cache, device, c.mixed, t)) {
        rep << "cached " << tuning_key(g, device, c.mixed);
        if (report) *report = rep.str();
        return group_set_tuning(g, t, st);
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int rc = FASTPI_OK;
    auto elapsed = [&](float& ms) -> bool {
        if (hipEventSynchronize(e1) != hipSuccess) return false;
        return hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    };
    Tuning best = g.tune;
    do {
        // one full run puts the gathered values in place for the block-SVD trials
        if ((rc = group_set_tuning(g, best, st)) != FASTPI_OK) break;
        if ((rc = group_svd(g, val, U, S, V, c)) != FASTPI_OK) break;
        // 1) block SVD: LDS budget and persistent occupancy
        const int cand_blk[][2] = {{16 * 1024, 8}, {32 * 1024, 4}, {56 * 1024, 2}};
        float best_ms = 1e30f;
        for (const auto& cb : cand_blk) {
            float tmin = 1e30f;
            for (int rep_i = 0; rep_i < 3; ++rep_i) {
                hipEventRecord(e0, st);
                launch_block_svd_tasks(c.mixed, g.tasks, g.ntasks, g.counter, cb[0], g.ncu * cb[1], c.max_sweeps,
                                       c.tol, st);
                hipEventRecord(e1, st);
                float ms = 0;
                if (!elapsed(ms)) {
                    rc = FASTPI_EHIP;
                    break;
                }
                tmin = std::min(tmin, ms);
            }
            if (rc != FASTPI_OK) break;
            rep << "block lds=" << cb[0] << " wgs/cu=" << cb[1] << " " << tmin << " ms; ";
            if (tmin < best_ms) {
                best_ms = tmin;
                best.block_lds = cb[0];
                best.block_wgs_per_cu = cb[1];
            }
        }
        if (rc != FASTPI_OK) break;
        // 2) eigensolver: partial-Gram height, inner sweeps and the preconditioner, timed
        // over whole runs (the inner sweeps and the start change the number of outer sweeps)
        best_ms = 1e30f;
        Tuning eig_best = best;
        const int cand_eig[][3] = {{64, 1, 1}, {128, 1, 1}, {256, 1, 1}, {128, 2, 1}, {128, 1, 0}, {64, 1, 0}};
        for (const auto& ce : cand_eig) {
            Tuning cand = best;
            cand.gram_rows = ce[0];
            cand.inner_sweeps = ce[1];
            cand.precond = ce[2];
            if ((rc = group_set_tuning(g, cand, st)) != FASTPI_OK) break;
            hipEventRecord(e0, st);
            if ((rc = group_svd(g, val, U, S, V, c)) != FASTPI_OK) break;
            hipEventRecord(e1, st);
            float ms = 0;
            if (!elapsed(ms)) {
                rc = FASTPI_EHIP;
                break;
            }
            rep << "eig rows=" << ce[0] << " inner=" << ce[1] << " precond=" << ce[2] << " " << ms << " ms; ";
            if (ms < best_ms) {
                best_ms = ms;
                eig_best = cand;
            }
        }
        if (rc != FASTPI_OK) break;
        best = eig_best;
        // 3) the core route: subspace iteration where it applies, or Jacobi on every core
        // (in a batch the Jacobi cores of all matrices share the eigensolver's launches, which
        // can outweigh the subspace route's smaller problems); timed only when it changes a route
        {
            const int other = g.core.mode == 1 ? 0 : 1;
            CoreCfg alt = g.core;
            alt.mode = other;
            bool changes = false;
            for (const Instance* I : g.inst) {
                const DevicePlan& d = I->dp;
                const bool a = core_basis(g.core, d.s, d.n1, g.mixed) > 0 ||
                               core_basis(g.core, d.r, d.s + d.n2, g.mixed) > 0;
                const bool b = core_basis(alt, d.s, d.n1, g.mixed) > 0 || core_basis(alt, d.r, d.s + d.n2, g.mixed) > 0;
                changes = changes || a != b;
            }
            best.core_mode = g.core.mode;
            if (changes) {
                Tuning cand = best;
                cand.core_mode = other;
                if ((rc = group_set_tuning(g, cand, st)) != FASTPI_OK) break;
                hipEventRecord(e0, st);
                if ((rc = group_svd(g, val, U, S, V, c)) != FASTPI_OK) break;
                hipEventRecord(e1, st);
                float ms = 0;
                if (!elapsed(ms)) {
                    rc = FASTPI_EHIP;
                    break;
                }
                rep << "core=" << other << " " << ms << " ms; ";
                if (ms < best_ms) {
                    best_ms = ms;
                    best = cand;
                }
            }
        }
        if ((rc = group_set_tuning(g, best, st)) != FASTPI_OK) break;
        rep << "chose lds=" << best.block_lds << " wgs/cu=" << best.block_wgs_per_cu << " rows=" << best.gram_rows
            << " inner=" << best.inner_sweeps << " precond=" << best.precond << " core=" << best.core_mode;
        if (cache) rc = store_tuning(g, cache, device, c.mixed, best);
    } while (false);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (report) *report = rep.str();
    return rc;
}

}  // namespace fastpi
