// C ABI: plans (host), handles and the device path of Algorithm 1 lines 2-5.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "host_internal.h"
#include "kernels.h"

namespace fastpi {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace fastpi

using namespace fastpi;

struct fastpi_plan {
    Plan p;
};

namespace {

template <typename T>
struct DevBuf {
    T* ptr = nullptr;
    size_t count = 0;
};

struct DevicePlan {
    bool valid = false;
    int64_t m = 0, n = 0, nnz = 0, m1 = 0, n1 = 0, m2 = 0, n2 = 0, s_b = 0, s = 0, r = 0;
    int64_t B_dense = 0, val_elems = 0, blk_elems = 0, u1 = 0, v1 = 0;
    int64_t off_a21r = 0, off_a21c = 0, off_tr = 0, off_tc = 0;
    int nbig = 0;             // work items too large for the small-LDS launch
    int64_t gscratch = 0;     // elements of global Jacobi scratch for the largest items
    BlockWork* work = nullptr;
    int64_t *dst0 = nullptr, *dst1 = nullptr, *gscratch_off = nullptr;
    int64_t *a21_rowptr = nullptr, *a21_colptr = nullptr, *t_rowptr = nullptr, *t_colptr = nullptr;
    int *a21_colidx = nullptr, *a21_rowidx = nullptr, *t_colidx = nullptr, *t_rowidx = nullptr;
    int *piT = nullptr, *invT = nullptr, *invF = nullptr;
    int2 *pairs2 = nullptr, *pairs3 = nullptr;
    SegDev seg_a21c{}, seg_a21r{}, seg_tc{}, seg_tr{};
};

constexpr int kSmallLds = 16 * 1024;
constexpr int kBigLds = 60 * 1024;

}  // namespace

struct fastpi_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t copy_stream = nullptr;   // side stream for reading convergence counters
    fastpi_options opts{};
    DevicePlan dp;
    std::vector<void*> plan_allocs;
    double* ws = nullptr;
    size_t ws_bytes = 0;
    int* iws = nullptr;
    size_t iws_bytes = 0;
    int* status = nullptr;       // device: [0] status bits, [1] block sweeps
    int* host_pinned = nullptr;  // pinned host words for the sweep counters
    int32_t sweeps[3] = {0, 0, 0};
    // offsets (in doubles) of the stage buffers inside ws
    int64_t o_vals, o_u1, o_v1, o_sig1, o_g2, o_v2, o_lam2, o_sig2, o_inv2, o_u2, o_g3, o_vt, o_lam3,
        o_sig3, o_inv3, o_c1, o_c2, o_eig, o_part, o_gs, o_spart, o_end;
    // apply scratch
    double* aws = nullptr;
    size_t aws_bytes = 0;
    KernelTimer timer;
    // rank-predictor scratch
    float* mws = nullptr;
    size_t mws_bytes = 0;
};

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

int check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("HIP launch error: ") + hipGetErrorString(e));
        return FASTPI_EHIP;
    }
    return FASTPI_OK;
}

template <typename T>
int upload(fastpi_handle* h, T*& dst, const T* src, size_t count) {
    dst = nullptr;
    if (count == 0) return FASTPI_OK;
    void* p = nullptr;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
        set_error("device allocation failed for a plan table");
        return FASTPI_ENOMEM;
    }
    h->plan_allocs.push_back(p);
    dst = static_cast<T*>(p);
    HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, h->stream));
    return FASTPI_OK;
}

void free_plan(fastpi_handle* h) {
    if (!h->plan_allocs.empty()) hipStreamSynchronize(h->stream);
    for (void* p : h->plan_allocs) hipFree(p);
    h->plan_allocs.clear();
    h->dp = DevicePlan{};
}

int ensure_ws(fastpi_handle* h, size_t bytes) {
    if (bytes <= h->ws_bytes) return FASTPI_OK;
    if (h->opts.max_workspace_bytes && bytes > h->opts.max_workspace_bytes) {
        set_error("workspace of " + std::to_string(bytes) + " bytes exceeds the cap");
        return FASTPI_ENOMEM;
    }
    if (h->ws) {
        hipStreamSynchronize(h->stream);
        hipFree(h->ws);
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        set_error("device workspace allocation of " + std::to_string(bytes) + " bytes failed");
        return FASTPI_ENOMEM;
    }
    h->ws = static_cast<double*>(p);
    h->ws_bytes = bytes;
    return FASTPI_OK;
}

int ensure_iws(fastpi_handle* h, size_t bytes) {
    if (bytes <= h->iws_bytes) return FASTPI_OK;
    if (h->iws) {
        hipStreamSynchronize(h->stream);
        hipFree(h->iws);
        h->iws = nullptr;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        set_error("device allocation failed (int workspace)");
        return FASTPI_ENOMEM;
    }
    h->iws = static_cast<int*>(p);
    h->iws_bytes = bytes;
    return FASTPI_OK;
}

int upload_segments(fastpi_handle* h, const Segments& s, SegDev& d) {
    int st;
    const int32_t* p32 = nullptr;
    const int64_t* p64 = nullptr;
    d = SegDev{};
    int32_t* owner = nullptr;
    int32_t* pidx = nullptr;
    int32_t* mo = nullptr;
    int32_t* mp = nullptr;
    int64_t* b = nullptr;
    int64_t* e = nullptr;
    (void)p32;
    (void)p64;
    if ((st = upload(h, owner, s.owner.data(), s.owner.size())) != FASTPI_OK) return st;
    if ((st = upload(h, pidx, s.pidx.data(), s.pidx.size())) != FASTPI_OK) return st;
    if ((st = upload(h, b, s.begin.data(), s.begin.size())) != FASTPI_OK) return st;
    if ((st = upload(h, e, s.end.data(), s.end.size())) != FASTPI_OK) return st;
    if ((st = upload(h, mo, s.multi_owner.data(), s.multi_owner.size())) != FASTPI_OK) return st;
    if ((st = upload(h, mp, s.multi_ptr.data(), s.multi_ptr.size())) != FASTPI_OK) return st;
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

int64_t eig_pairs_count(int64_t q) {
    std::vector<int2> t;
    eig_pair_table(q, t);
    return static_cast<int64_t>(t.size());
}

}  // namespace

extern "C" {

const char* fastpi_last_error(void) { return g_last_error.c_str(); }

int64_t fastpi_target_rank(double alpha, int64_t x) { return target_rank(alpha, x); }

int fastpi_reorder(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col,
                   const double* val, double k, int32_t* piT, int32_t* piF, int64_t* blocks,
                   int64_t blocks_cap, int64_t* num_blocks, fastpi_split* out) {
    if (!piT || !piF || !num_blocks) {
        set_error("null output pointer");
        return FASTPI_EINVAL;
    }
    int st = validate_csr(m, n, rowptr, col, val);
    if (st != FASTPI_OK) return st;
    ReorderOut ro;
    st = reorder_pattern(m, n, rowptr, col, val, k, ro);
    if (st != FASTPI_OK) return st;
    const int64_t B = static_cast<int64_t>(ro.blocks.size());
    *num_blocks = B;
    if (blocks_cap > 0 && blocks_cap < B) {
        set_error("block buffer too small");
        return FASTPI_EINVAL;
    }
    std::memcpy(piT, ro.piT.data(), sizeof(int32_t) * m);
    std::memcpy(piF, ro.piF.data(), sizeof(int32_t) * n);
    if (blocks && blocks_cap >= B) {
        for (int64_t b = 0; b < B; ++b) {
            blocks[4 * b + 0] = ro.blocks[b].row0;
            blocks[4 * b + 1] = ro.blocks[b].col0;
            blocks[4 * b + 2] = ro.blocks[b].rows;
            blocks[4 * b + 3] = ro.blocks[b].cols;
        }
    }
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->m = m;
        out->n = n;
        out->nnz = ro.nnz_edges;
        out->m1 = ro.m1;
        out->n1 = ro.n1;
        out->m2 = ro.m2;
        out->n2 = ro.n2;
        out->B = B;
        int64_t bd = 0;
        for (const auto& d : ro.blocks) bd += (d.rows > 0 && d.cols > 0);
        out->B_dense = bd;
        out->T_it = ro.iterations;
    }
    return FASTPI_OK;
}

int fastpi_plan_create(fastpi_plan** plan, int64_t m, int64_t n, const int64_t* rowptr,
                       const int32_t* col, const double* val, double alpha, double k) {
    if (!plan) {
        set_error("null plan pointer");
        return FASTPI_EINVAL;
    }
    *plan = nullptr;
    fastpi_plan* p = new (std::nothrow) fastpi_plan();
    if (!p) {
        set_error("host allocation failed");
        return FASTPI_ENOMEM;
    }
    int st = build_plan(p->p, m, n, rowptr, col, val, alpha, k);
    if (st != FASTPI_OK) {
        delete p;
        return st;
    }
    *plan = p;
    return FASTPI_OK;
}

int fastpi_plan_info(const fastpi_plan* plan, fastpi_split* out) {
    if (!plan || !out) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    const Plan& p = plan->p;
    std::memset(out, 0, sizeof(*out));
    out->m = p.m;
    out->n = p.n;
    out->nnz = p.ro.nnz_edges;
    out->m1 = p.ro.m1;
    out->n1 = p.ro.n1;
    out->m2 = p.ro.m2;
    out->n2 = p.ro.n2;
    out->B = static_cast<int64_t>(p.ro.blocks.size());
    out->B_dense = p.B_dense;
    out->T_it = p.ro.iterations;
    out->s_b = p.s_b;
    out->s = p.s;
    out->r = p.r;
    return FASTPI_OK;
}

int fastpi_plan_permutation(const fastpi_plan* plan, int32_t* piT, int32_t* piF) {
    if (!plan) {
        set_error("null plan");
        return FASTPI_EINVAL;
    }
    if (piT) std::memcpy(piT, plan->p.ro.piT.data(), sizeof(int32_t) * plan->p.m);
    if (piF) std::memcpy(piF, plan->p.ro.piF.data(), sizeof(int32_t) * plan->p.n);
    return FASTPI_OK;
}

int fastpi_plan_blocks(const fastpi_plan* plan, int64_t* blocks) {
    if (!plan || !blocks) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    const auto& B = plan->p.ro.blocks;
    for (size_t b = 0; b < B.size(); ++b) {
        blocks[4 * b + 0] = B[b].row0;
        blocks[4 * b + 1] = B[b].col0;
        blocks[4 * b + 2] = B[b].rows;
        blocks[4 * b + 3] = B[b].cols;
    }
    return FASTPI_OK;
}

int fastpi_plan_block_ranks(const fastpi_plan* plan, int64_t* ranks) {
    if (!plan || !ranks) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    std::memcpy(ranks, plan->p.block_rank.data(), sizeof(int64_t) * plan->p.block_rank.size());
    return FASTPI_OK;
}

void fastpi_plan_destroy(fastpi_plan* plan) { delete plan; }

int fastpi_create(fastpi_handle** h, int device, void* hip_stream, const fastpi_options* opts) {
    if (!h) {
        set_error("null handle pointer");
        return FASTPI_EINVAL;
    }
    *h = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) {
        set_error("device index out of range");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(device));
    fastpi_handle* H = new (std::nothrow) fastpi_handle();
    if (!H) {
        set_error("host allocation failed");
        return FASTPI_ENOMEM;
    }
    H->device = device;
    H->stream = static_cast<hipStream_t>(hip_stream);
    if (opts) H->opts = *opts;
    if (H->opts.max_sweeps <= 0) H->opts.max_sweeps = 60;
    void* p = nullptr;
    if (hipMalloc(&p, 64) != hipSuccess) {
        delete H;
        set_error("device allocation failed");
        return FASTPI_ENOMEM;
    }
    H->status = static_cast<int*>(p);
    if (hipHostMalloc(&p, 64, hipHostMallocDefault) != hipSuccess) {
        hipFree(H->status);
        delete H;
        set_error("pinned host allocation failed");
        return FASTPI_ENOMEM;
    }
    H->host_pinned = static_cast<int*>(p);
    if (hipStreamCreateWithFlags(&H->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        hipFree(H->status);
        hipHostFree(H->host_pinned);
        delete H;
        set_error("stream creation failed");
        return FASTPI_EHIP;
    }
    launch_fill_i32(H->status, 16, 0, H->stream);
    *h = H;
    return check_launch();
}

int fastpi_set_precision(fastpi_handle* h, fastpi_precision p) {
    if (!h || (p != FASTPI_FP64 && p != FASTPI_MIXED)) {
        set_error("bad handle or precision");
        return FASTPI_EINVAL;
    }
    h->opts.precision = p;
    return FASTPI_OK;
}

void fastpi_destroy(fastpi_handle* h) {
    if (!h) return;
    hipSetDevice(h->device);
    hipStreamSynchronize(h->stream);
    free_plan(h);
    if (h->ws) hipFree(h->ws);
    if (h->iws) hipFree(h->iws);
    if (h->aws) hipFree(h->aws);
    if (h->mws) hipFree(h->mws);
    if (h->status) hipFree(h->status);
    if (h->host_pinned) hipHostFree(h->host_pinned);
    if (h->copy_stream) hipStreamDestroy(h->copy_stream);
    for (hipEvent_t e : h->timer.pool) hipEventDestroy(e);
    delete h;
}

int fastpi_upload_plan(fastpi_handle* h, const fastpi_plan* plan) {
    if (!h || !plan) {
        set_error("null handle or plan");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    free_plan(h);
    const Plan& p = plan->p;
    DevicePlan& d = h->dp;
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
    // work items needing more LDS than the small launch offers come first (cost order)
    std::vector<int64_t> goff(p.work.size(), 0);
    int nbig = 0;
    int64_t gs = 0;
    for (size_t i = 0; i < p.work.size(); ++i) {
        const BlockWork& w = p.work[i];
        const int64_t pp = std::max(w.rows, w.cols), qq = std::min(w.rows, w.cols);
        const int64_t need = pp * qq + qq * qq;
        if (qq > 256) {
            set_error("a diagonal block has both sides above 256; not supported");
            return FASTPI_EINTERNAL;
        }
        if (need * static_cast<int64_t>(sizeof(double)) > kSmallLds) nbig = static_cast<int>(i) + 1;
        if (need * static_cast<int64_t>(sizeof(double)) > kBigLds) {
            goff[i] = gs;
            gs += need;
        }
    }
    d.nbig = nbig;
    d.gscratch = gs;
    int st;
    if ((st = upload(h, d.work, p.work.data(), p.work.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.gscratch_off, goff.data(), goff.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.dst0, p.dst0.data(), p.dst0.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.dst1, p.dst1.data(), p.dst1.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.a21_rowptr, p.a21_rowptr.data(), p.a21_rowptr.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.a21_colptr, p.a21_colptr.data(), p.a21_colptr.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.t_rowptr, p.t_rowptr.data(), p.t_rowptr.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.t_colptr, p.t_colptr.data(), p.t_colptr.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.a21_colidx, p.a21_colidx.data(), p.a21_colidx.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.a21_rowidx, p.a21_rowidx.data(), p.a21_rowidx.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.t_colidx, p.t_colidx.data(), p.t_colidx.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.t_rowidx, p.t_rowidx.data(), p.t_rowidx.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.piT, p.ro.piT.data(), p.ro.piT.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.invF, p.invF.data(), p.invF.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.invT, p.invT.data(), p.invT.size())) != FASTPI_OK) return st;
    if ((st = upload_segments(h, p.seg_a21c, d.seg_a21c)) != FASTPI_OK) return st;
    if ((st = upload_segments(h, p.seg_a21r, d.seg_a21r)) != FASTPI_OK) return st;
    if ((st = upload_segments(h, p.seg_tc, d.seg_tc)) != FASTPI_OK) return st;
    if ((st = upload_segments(h, p.seg_tr, d.seg_tr)) != FASTPI_OK) return st;
    std::vector<int2> t2, t3;
    if (d.n1 > 0) eig_pair_table(d.n1, t2);
    const int64_t q3 = d.s + d.n2;
    if (q3 > 0) eig_pair_table(q3, t3);
    if ((st = upload(h, d.pairs2, t2.data(), t2.size())) != FASTPI_OK) return st;
    if ((st = upload(h, d.pairs3, t3.data(), t3.size())) != FASTPI_OK) return st;

    // workspace layout (doubles)
    const int64_t m = d.m, n1 = d.n1, n2 = d.n2, s = d.s, r = d.r;
    int64_t o = 0;
    auto take = [&o](int64_t cnt) {
        const int64_t at = o;
        o += ((cnt + 31) / 32) * 32;
        return at;
    };
    h->o_vals = take(d.val_elems);
    h->o_u1 = take(d.u1);
    h->o_v1 = take(d.v1);
    h->o_sig1 = take(d.s_b);
    h->o_g2 = take(n1 * n1);
    h->o_v2 = take(n1 * s);
    h->o_lam2 = take(s);
    h->o_sig2 = take(s);
    h->o_inv2 = take(s);
    h->o_u2 = take(m * s);
    h->o_g3 = take(q3 * q3);
    h->o_vt = take(q3 * r);
    h->o_lam3 = take(r);
    h->o_sig3 = take(r);
    h->o_inv3 = take(r);
    h->o_c1 = take(s * r);
    h->o_c2 = take(n2 * r);
    h->o_eig = take(static_cast<int64_t>(std::max(eig_workspace_doubles(std::max<int64_t>(n1, 1)),
                                                  eig_workspace_doubles(std::max<int64_t>(q3, 1)))));
    const int sp = gemm_tn_splits(s, s, m);
    h->o_part = take(static_cast<int64_t>(sp) * s * s);
    h->o_gs = take(gs);
    const int64_t spart = std::max({p.seg_a21c.npart * n1, p.seg_tc.npart * std::max(n2, s),
                                    p.seg_a21r.npart * s, p.seg_tr.npart * r, int64_t(1)});
    h->o_spart = take(spart);
    h->o_end = o;
    st = ensure_ws(h, static_cast<size_t>(o) * sizeof(double));
    if (st != FASTPI_OK) return st;
    st = ensure_iws(h, std::max(eig_int_workspace(std::max<int64_t>(n1, 1), h->opts.max_sweeps),
                                eig_int_workspace(std::max<int64_t>(q3, 1), h->opts.max_sweeps)) * sizeof(int));
    if (st != FASTPI_OK) return st;
    d.valid = true;
    return check_launch();
}

int fastpi_svd(fastpi_handle* h, const int64_t* rowptr, const int32_t* col, const double* val,
               double* U, double* S, double* V) {
    (void)rowptr;
    (void)col;
    if (!h || !h->dp.valid) {
        set_error("no plan uploaded to this handle");
        return FASTPI_EINVAL;
    }
    const DevicePlan& d = h->dp;
    if ((!val && d.nnz > 0) || (!U && d.m * d.r > 0) || (!S && d.r > 0) || (!V && d.n * d.r > 0)) {
        set_error("null device pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    hipStream_t st = h->stream;
    double* ws = h->ws;
    const bool mixed = h->opts.precision == FASTPI_MIXED;
    const int64_t m = d.m, n1 = d.n1, m1 = d.m1, m2 = d.m2, n2 = d.n2, s = d.s, r = d.r;
    const int64_t q3 = s + n2;
    double* vals = ws + h->o_vals;
    double* U1 = ws + h->o_u1;
    double* V1 = ws + h->o_v1;
    double* sig1 = ws + h->o_sig1;
    double* G2 = ws + h->o_g2;
    double* V2 = ws + h->o_v2;
    double* lam2 = ws + h->o_lam2;
    double* sig2 = ws + h->o_sig2;
    double* inv2 = ws + h->o_inv2;
    double* U2 = ws + h->o_u2;
    double* G3 = ws + h->o_g3;
    double* Vt = ws + h->o_vt;
    double* lam3 = ws + h->o_lam3;
    double* sig3 = ws + h->o_sig3;
    double* inv3 = ws + h->o_inv3;
    double* C1 = ws + h->o_c1;
    double* C2 = ws + h->o_c2;
    double* eigws = ws + h->o_eig;
    double* part = ws + h->o_part;
    double* gsc = ws + h->o_gs;
    double* spart = ws + h->o_spart;
    const double tol = h->opts.tol;
    const int max_sweeps = h->opts.max_sweeps;
    // Singular values below this fraction of the largest are not resolved by the Gram route
    // (about sqrt(q eps)); they are returned as zero.
    const double rel_cut = 1e-7;
    int rc;

    launch_fill_i32(h->status, 2, 0, st);
    // a1: split the reordered matrix into dense A11 blocks, A21 and T
    launch_fill(vals, d.blk_elems, 0.0, st);
    launch_gather(val, d.dst0, d.dst1, d.nnz, vals, h->status, st);
    // a2: block SVDs (Eq. 1)
    {
        const long ts = h->timer.begin(KT_BLOCK_SVD, st);
        launch_block_svd(mixed, d.work, 0, d.nbig, vals, gsc, d.gscratch_off, kBigLds, U1, sig1, V1,
                         max_sweeps, tol, h->status + 1, h->status, st);
        launch_block_svd(mixed, d.work, d.nbig, static_cast<int>(d.B_dense - d.nbig), vals, gsc,
                         d.gscratch_off, kSmallLds, U1, sig1, V1, max_sweeps, tol, h->status + 1,
                         h->status, st);
        h->timer.end(ts, st);
    }
    // a3: row update (Eq. 2) -- top s eigenpairs of M2^T M2 = V1 Sigma1^2 V1^T + A21^T A21
    if (n1 > 0 && s > 0) {
        launch_fill(G2, n1 * n1, 0.0, st);
        launch_blockdiag_gram(d.work, static_cast<int>(d.B_dense), V1, sig1, G2, n1, st);
        launch_sparse_gram(d.seg_a21c, d.a21_rowidx, vals + d.off_a21c, d.a21_rowptr, d.a21_colidx,
                           vals + d.off_a21r, n1, G2, n1, true, spart, st);
        rc = eig_top(G2, n1, s, lam2, V2, eigws, h->iws, d.pairs2, max_sweeps, 0.0, 1,
                     &h->sweeps[1], h->host_pinned, st, h->copy_stream, &h->timer);
        if (rc != FASTPI_OK && rc != FASTPI_ENOCONV) return rc;
        if (rc == FASTPI_ENOCONV) launch_fill_i32(h->status, 1, 2, st);
        launch_sqrt_inv(lam2, s, rel_cut, sig2, inv2, st);
        launch_fill(U2, m * s, 0.0, st);
        launch_u2_top(d.work, static_cast<int>(d.B_dense), U1, sig1, V1, V2, s, inv2, U2, h->status, st);
        launch_spmm_rows(d.seg_a21r, d.a21_colidx, vals + d.off_a21r, V2, s, inv2, U2 + m1 * s, s,
                         nullptr, false, spart, st);
    }
    // a4: column update (Eq. 3) -- top r eigenpairs of X3^T X3, X3 = [U2 Sigma2, T]
    if (q3 > 0 && r > 0) {
        launch_fill(G3, q3 * q3, 0.0, st);
        if (s > 0) {
            const int sp = gemm_tn_splits(s, s, m);
            launch_gemm_tn(U2, s, U2, s, s, s, m, G3, q3, sig2, sig2, part, sp, st, mixed);
            launch_sparse_proj(d.seg_tc, d.t_rowidx, vals + d.off_tc, U2, s, sig2, G3, q3, s, spart, st);
        }
        launch_sparse_gram(d.seg_tc, d.t_rowidx, vals + d.off_tc, d.t_rowptr, d.t_colidx,
                           vals + d.off_tr, n2, G3 + s * q3 + s, q3, false, spart, st);
        rc = eig_top(G3, q3, r, lam3, Vt, eigws, h->iws, d.pairs3, max_sweeps, 0.0, 1, &h->sweeps[2],
                     h->host_pinned, st, h->copy_stream, &h->timer);
        if (rc != FASTPI_OK && rc != FASTPI_ENOCONV) return rc;
        if (rc == FASTPI_ENOCONV) launch_fill_i32(h->status, 1, 2, st);
        launch_sqrt_inv(lam3, r, rel_cut, sig3, inv3, st);
        launch_col_coeffs(Vt, s, n2, r, sig2, inv3, C1, C2, st);
        // a5: U and V in the caller's order
        launch_gemm_nn(U2, s, d.piT, C1, r, m, r, s, U, r, nullptr, st, mixed);
        launch_spmm_rows(d.seg_tr, d.t_colidx, vals + d.off_tr, C2, r, nullptr, U, r, d.invT, true,
                         spart, st);
        launch_gemm_nn(V2, s, nullptr, Vt, r, n1, r, s, V, r, d.invF, st, mixed);
        launch_copy_rows(Vt + s * r, n2, r, d.invF + n1, V, st);
        HIP_TRY(hipMemcpyAsync(S, sig3, sizeof(double) * r, hipMemcpyDeviceToDevice, st));
    }
    return check_launch();
}

int fastpi_apply(fastpi_handle* h, int64_t m, int64_t n, int64_t r, const double* U,
                 const double* S, const double* V, int64_t L, const double* Y, double* Z) {
    if (!h || m <= 0 || n <= 0 || r < 0 || L < 0) {
        set_error("bad handle or sizes");
        return FASTPI_EINVAL;
    }
    if (r == 0 || L == 0) return FASTPI_OK;
    if (!U || !S || !V || !Y || !Z) {
        set_error("null device pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    hipStream_t st = h->stream;
    const int sp = gemm_tn_splits(r, L, m);
    const size_t need = static_cast<size_t>(r + r * L + static_cast<int64_t>(sp) * r * L) * sizeof(double);
    if (need > h->aws_bytes) {
        if (h->aws) {
            hipStreamSynchronize(st);
            hipFree(h->aws);
            h->aws = nullptr;
            h->aws_bytes = 0;
        }
        void* p = nullptr;
        if (hipMalloc(&p, need) != hipSuccess) {
            set_error("device allocation failed (apply scratch)");
            return FASTPI_ENOMEM;
        }
        h->aws = static_cast<double*>(p);
        h->aws_bytes = need;
    }
    double* inv = h->aws;
    double* W = inv + r;
    double* part = W + r * L;
    launch_pinv_sigma(S, r, static_cast<double>(std::max(m, n)) * DBL_EPSILON, inv, st);
    const bool mixed = h->opts.precision == FASTPI_MIXED;
    launch_gemm_tn(U, r, Y, L, r, L, m, W, L, inv, nullptr, part, sp, st, mixed);
    launch_gemm_nn(V, r, nullptr, W, L, n, L, r, Z, L, nullptr, st, mixed);
    return check_launch();
}

int fastpi_stage_output(fastpi_handle* h, int which, double* dst, int64_t count) {
    if (!h || !h->dp.valid || !dst) {
        set_error("bad handle or pointer");
        return FASTPI_EINVAL;
    }
    const DevicePlan& d = h->dp;
    const double* src = nullptr;
    int64_t want = 0;
    switch (which) {
        case 0: src = h->ws + h->o_sig1; want = d.s_b; break;
        case 1: src = h->ws + h->o_sig2; want = d.s; break;
        case 2: src = h->ws + h->o_v2; want = d.n1 * d.s; break;
        case 3: src = h->ws + h->o_u2; want = d.m * d.s; break;
        default: set_error("unknown stage"); return FASTPI_EINVAL;
    }
    if (count != want) {
        set_error("stage size mismatch: expected " + std::to_string(want));
        return FASTPI_EINVAL;
    }
    if (want > 0)
        HIP_TRY(hipMemcpyAsync(dst, src, sizeof(double) * want, hipMemcpyDeviceToDevice, h->stream));
    return FASTPI_OK;
}

int fastpi_syev_top(fastpi_handle* h, int64_t q, const double* G, int64_t t, double* vals,
                    double* vecs) {
    if (!h || q <= 0 || t <= 0 || t > q || !G || !vals || !vecs) {
        set_error("bad arguments");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    // the eigensolver needs its own workspace; use the plan workspace when none is uploaded
    const size_t need = eig_workspace_doubles(q) * sizeof(double);
    int st = FASTPI_OK;
    if (h->dp.valid) {
        if (need > static_cast<size_t>(h->o_end - h->o_eig) * sizeof(double)) {
            set_error("eigensolver order exceeds the uploaded plan's workspace");
            return FASTPI_EINVAL;
        }
    } else if ((st = ensure_ws(h, need)) != FASTPI_OK) {
        return st;
    }
    double* ws = h->dp.valid ? h->ws + h->o_eig : h->ws;
    if ((st = ensure_iws(h, eig_int_workspace(q, h->opts.max_sweeps) * sizeof(int))) != FASTPI_OK) return st;
    std::vector<int2> tab;
    eig_pair_table(q, tab);
    void* p = nullptr;
    if (hipMalloc(&p, tab.size() * sizeof(int2)) != hipSuccess) {
        set_error("device allocation failed (pair table)");
        return FASTPI_ENOMEM;
    }
    HIP_TRY(hipMemcpyAsync(p, tab.data(), tab.size() * sizeof(int2), hipMemcpyHostToDevice, h->stream));
    int sw = 0;
    st = eig_top(G, q, t, vals, vecs, ws, h->iws, static_cast<int2*>(p), h->opts.max_sweeps,
                 h->opts.tol, 1, &sw, h->host_pinned, h->stream, h->copy_stream, &h->timer);
    hipStreamSynchronize(h->stream);
    hipFree(p);
    h->sweeps[1] = sw;
    if (st != FASTPI_OK) {
        if (st == FASTPI_ENOCONV) set_error("eigensolver reached the sweep cap");
        return st;
    }
    return check_launch();
}

int fastpi_sync(fastpi_handle* h) {
    if (!h) {
        set_error("null handle");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(hipMemcpyAsync(h->host_pinned, h->status, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const int bits = h->host_pinned[0];
    h->sweeps[0] = h->host_pinned[1];
    if (bits & 1) {
        set_error("non-finite value in A");
        return FASTPI_ENONFINITE;
    }
    if (bits & 2) {
        set_error("a Jacobi iteration reached its sweep cap");
        return FASTPI_ENOCONV;
    }
    if (bits & 4) {
        set_error("internal: block rank above the supported bound");
        return FASTPI_EINTERNAL;
    }
    return FASTPI_OK;
}

int fastpi_block_features(const fastpi_plan* plan, const double* val, double* out) {
    if (!plan || !val || !out) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    return block_features(plan->p, val, out);
}

int fastpi_plan_set_block_ranks(fastpi_plan* plan, const int64_t* ranks) {
    if (!plan || !ranks) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    const size_t B = plan->p.ro.blocks.size();
    std::vector<int64_t> r(ranks, ranks + B);
    for (int64_t v : r)
        if (v < 0) {
            set_error("negative block rank");
            return FASTPI_EINVAL;
        }
    assign_ranks(plan->p, r);
    return FASTPI_OK;
}

int fastpi_mlp_param_count(void) { return mlp_param_count(); }

int fastpi_mlp_forward(fastpi_handle* h, int64_t N, const float* X, const float* theta, float* f) {
    if (!h || N < 0 || (N > 0 && (!X || !theta || !f))) {
        set_error("bad arguments");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    launch_mlp_forward(N, X, theta, f, nullptr, h->stream);
    return check_launch();
}

int fastpi_mlp_gradient(fastpi_handle* h, int64_t N, const float* X, const float* y,
                        const float* theta, float* grad) {
    if (!h || N <= 0 || !X || !y || !theta || !grad) {
        set_error("bad arguments");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    const size_t need = mlp_scratch_floats(N) * sizeof(float);
    if (need > h->mws_bytes) {
        if (h->mws) {
            hipStreamSynchronize(h->stream);
            hipFree(h->mws);
            h->mws = nullptr;
            h->mws_bytes = 0;
        }
        void* p = nullptr;
        if (hipMalloc(&p, need) != hipSuccess) {
            set_error("device allocation failed (rank-predictor scratch)");
            return FASTPI_ENOMEM;
        }
        h->mws = static_cast<float*>(p);
        h->mws_bytes = need;
    }
    launch_mlp_gradient(N, X, y, theta, grad, h->mws, h->stream);
    return check_launch();
}

int fastpi_mlp_adam(fastpi_handle* h, float* theta, const float* grad, float* m, float* v,
                    int64_t step, float lr) {
    if (!h || !theta || !grad || !m || !v || step < 1) {
        set_error("bad arguments");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    launch_mlp_adam(theta, grad, m, v, step, lr, h->stream);
    return check_launch();
}

int fastpi_timing_start(fastpi_handle* h, int kind) {
    if (!h || kind < KT_NONE || kind > KT_BLOCK_SVD) {
        set_error("bad handle or kernel kind");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->timer.target = kind;
    h->timer.used = 0;
    h->timer.failed = false;
    return FASTPI_OK;
}

int fastpi_timing_read(fastpi_handle* h, int64_t* launches, double* total_ms) {
    if (!h || !launches || !total_ms) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (h->timer.failed) {
        set_error("event creation failed while timing");
        return FASTPI_EHIP;
    }
    double tot = 0;
    const size_t pairs = h->timer.used / 2;
    for (size_t k = 0; k < pairs; ++k) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, h->timer.pool[2 * k], h->timer.pool[2 * k + 1]));
        tot += ms;
    }
    *launches = static_cast<int64_t>(pairs);
    *total_ms = tot;
    h->timer.used = 0;
    return FASTPI_OK;
}

int fastpi_last_sweeps(fastpi_handle* h, int32_t* out3) {
    if (!h || !out3) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    int st = fastpi_sync(h);
    for (int i = 0; i < 3; ++i) out3[i] = h->sweeps[i];
    return st;
}

}  // extern "C"
