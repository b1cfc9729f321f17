// C ABI: plans (host), handles, batches and the device path of Algorithm 1 lines 2-5.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <queue>
#include <vector>

#include "driver.h"
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

struct fastpi_handle {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t copy_stream = nullptr;   // side stream for reading convergence state
    fastpi_options opts{};
    Instance inst;                       // the uploaded plan
    Group grp;                           // a group of one: inst
    bool use_graph = false;
    std::string tune_cache;
    int* status = nullptr;       // device: [0] status bits, [1] block sweeps
    int* host_pinned = nullptr;  // pinned host words for the status read
    // apply scratch
    double* aws = nullptr;
    size_t aws_bytes = 0;
    // eigensolver scratch of fastpi_syev_top
    double* sws = nullptr;
    size_t sws_bytes = 0;
    int* siws = nullptr;
    size_t siws_bytes = 0;
    double* sa = nullptr;        // its pivoted-Cholesky scratch (the caller's G stays intact)
    size_t sa_bytes = 0;
    int32_t syev_sweeps = 0;
    KernelTimer timer;
    // rank-predictor scratch
    float* mws = nullptr;
    size_t mws_bytes = 0;
    // evaluation scratch (scores beyond the LDS capacity)
    double* ews = nullptr;
    size_t ews_bytes = 0;
    // batches created on this handle and not destroyed yet: released (and detached) when the
    // handle is destroyed first, so the two may be destroyed in either order
    std::vector<fastpi_batch*> batches;
};

// A sparse label matrix Y (m x L) held on the device as its transpose in CSR (per label,
// the rows where it is positive, with their values) and a segment table over labels.
struct fastpi_labels {
    int device = 0;
    int64_t m = 0, L = 0, nnz = 0;
    int32_t* rows = nullptr;   // device, per label in increasing row order
    double* vals = nullptr;
    SegDev seg{};
    // row-blocked form of the label SpMM (when no row has more than kLabelBlockPos positives):
    // the labelled rows in blocks, each block's positives by (sub-label, row)
    bool blocked = false;
    LabelBlocks lb;
    std::vector<void*> allocs;
};


struct fastpi_batch {
    fastpi_handle* h = nullptr;   // null once the handle was destroyed (the batch is detached)
    std::vector<Instance> inst;
    Group grp;
    int* status = nullptr;        // device: 2 words per instance
    int* host_status = nullptr;   // pinned mirror
    bool use_graph = false;
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
int grow(T*& buf, size_t& have, size_t bytes, hipStream_t st, const char* what) {
    if (bytes <= have) return FASTPI_OK;
    if (buf) {
        hipStreamSynchronize(st);
        hipFree(buf);
        buf = nullptr;
        have = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        set_error(std::string("device allocation failed (") + what + ")");
        return FASTPI_ENOMEM;
    }
    buf = static_cast<T*>(p);
    have = bytes;
    return FASTPI_OK;
}

// status bits of one instance -> status code (message set)
int decode_status(int bits) {
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
    if (bits & kStatusFloor) {
        set_error("warning: a kept singular value was at or below the Gram floor (1e-7 of the largest) "
                  "and is returned as 0");
        return FASTPI_WFLOOR;
    }
    return FASTPI_OK;
}

RunCfg run_cfg(fastpi_handle* h, bool use_graph) {
    RunCfg c;
    c.st = h->stream;
    c.copy_st = h->copy_stream;
    c.timer = use_graph ? nullptr : &h->timer;
    c.mixed = h->opts.precision == FASTPI_MIXED;
    c.max_sweeps = h->opts.max_sweeps;
    c.tol = h->opts.tol;
    c.use_graph = use_graph;
    return c;
}

Tuning from_c(const fastpi_tuning& t) {
    Tuning o;
    o.block_lds = t.block_lds;
    o.block_wgs_per_cu = t.block_wgs_per_cu;
    o.gram_rows = t.gram_rows;
    o.inner_sweeps = t.inner_sweeps;
    o.precond = t.precond;
    o.eig_fused = t.eig_fused;
    return o;
}

void to_c(const Tuning& t, fastpi_tuning* o) {
    o->block_lds = t.block_lds;
    o->block_wgs_per_cu = t.block_wgs_per_cu;
    o->gram_rows = t.gram_rows;
    o->inner_sweeps = t.inner_sweeps;
    o->precond = t.precond;
    o->eig_fused = t.eig_fused;
}

void copy_report(const std::string& rep, char* out, int64_t cap) {
    if (!out || cap <= 0) return;
    const size_t n = std::min<size_t>(rep.size(), static_cast<size_t>(cap - 1));
    std::memcpy(out, rep.data(), n);
    out[n] = '\0';
}

}  // namespace

extern "C" {

const char* fastpi_last_error(void) { return g_last_error.c_str(); }

int64_t fastpi_target_rank(double alpha, int64_t x) { return target_rank(alpha, x); }

// piT, piF, blocks and the shape report of a reordering into the caller's host buffers
static int reorder_outputs(const ReorderOut& ro, int64_t m, int64_t n, int32_t* piT, int32_t* piF, int64_t* blocks,
                           int64_t blocks_cap, int64_t* num_blocks, fastpi_split* out) {
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
    return reorder_outputs(ro, m, n, piT, piF, blocks, blocks_cap, num_blocks, out);
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

int fastpi_reorder_gpu(fastpi_handle* h, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                       const int32_t* col, const double* val, double k, int32_t* piT, int32_t* piF,
                       int64_t* blocks, int64_t blocks_cap, int64_t* num_blocks, fastpi_split* out) {
    if (!h || !piT || !piF || !num_blocks) {
        set_error("null handle or output pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    int st = validate_csr_gpu(m, n, nnz, rowptr, col, val, h->stream);
    if (st != FASTPI_OK) return st;
    ReorderOut ro;
    st = reorder_pattern_gpu(m, n, rowptr, col, val, nnz, k, h->stream, ro);
    if (st != FASTPI_OK) return st;
    return reorder_outputs(ro, m, n, piT, piF, blocks, blocks_cap, num_blocks, out);
}

int fastpi_plan_create_gpu(fastpi_plan** plan, fastpi_handle* h, int64_t m, int64_t n, const int64_t* rowptr,
                           const int32_t* col, const double* val, double alpha, double k) {
    if (!plan || !h) {
        set_error("null plan pointer or handle");
        return FASTPI_EINVAL;
    }
    *plan = nullptr;
    int st = validate_csr(m, n, rowptr, col, val);
    if (st != FASTPI_OK) return st;
    if (!(alpha > 0.0 && alpha <= 1.0)) {
        set_error("alpha must lie in (0, 1]");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    const int64_t nnz = rowptr[m];
    // the pattern (and values, for the stored-zero rule) on the device for the reordering
    std::vector<void*> bufs;
    auto cleanup = [&]() {
        hipStreamSynchronize(h->stream);
        for (void* p : bufs) hipFree(p);
    };
    auto dev_copy = [&](const void* src, size_t bytes) -> void* {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 1)) != hipSuccess) return nullptr;
        bufs.push_back(p);
        if (bytes && hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, h->stream) != hipSuccess) return nullptr;
        return p;
    };
    auto* drp = static_cast<int64_t*>(dev_copy(rowptr, sizeof(int64_t) * (m + 1)));
    auto* dcol = static_cast<int32_t*>(dev_copy(col, sizeof(int32_t) * nnz));
    double* dval = val ? static_cast<double*>(dev_copy(val, sizeof(double) * nnz)) : nullptr;
    if (!drp || !dcol || (val && !dval)) {
        cleanup();
        set_error("device allocation or copy failed (GPU reordering)");
        return FASTPI_ENOMEM;
    }
    ReorderOut ro;
    st = reorder_pattern_gpu(m, n, drp, dcol, dval, nnz, k, h->stream, ro);
    cleanup();
    if (st != FASTPI_OK) return st;
    fastpi_plan* p = new (std::nothrow) fastpi_plan();
    if (!p) {
        set_error("host allocation failed");
        return FASTPI_ENOMEM;
    }
    st = build_plan(p->p, m, n, rowptr, col, val, alpha, k, &ro);
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
    H->inst.status = H->status;
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

static void batch_release(fastpi_batch* b);
static bool batch_live(const fastpi_batch* b);

void fastpi_destroy(fastpi_handle* h) {
    if (!h) return;
    hipSetDevice(h->device);
    hipStreamSynchronize(h->stream);
    // release the device resources of the batches still alive on this handle; their host
    // objects stay valid (detached) until fastpi_batch_destroy
    for (fastpi_batch* b : h->batches) {
        batch_release(b);
        b->h = nullptr;
    }
    h->batches.clear();
    group_free(h->grp);
    instance_free(h->inst, h->stream);
    if (h->aws) hipFree(h->aws);
    if (h->sws) hipFree(h->sws);
    if (h->siws) hipFree(h->siws);
    if (h->sa) hipFree(h->sa);
    if (h->mws) hipFree(h->mws);
    if (h->ews) hipFree(h->ews);
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
    HIP_TRY(hipStreamSynchronize(h->stream));
    group_free(h->grp);
    int st = instance_upload(h->inst, plan->p, h->opts.max_workspace_bytes, h->stream);
    if (st != FASTPI_OK) return st;
    h->grp.inst = {&h->inst};
    h->grp.eig_tol = h->opts.tol;
    h->grp.mixed = h->opts.precision == FASTPI_MIXED;
    if ((st = group_build(h->grp, h->device, h->stream)) != FASTPI_OK) return st;
    Tuning t;
    if (!h->tune_cache.empty() &&
        tuning_lookup(h->grp, h->tune_cache.c_str(), h->device, h->opts.precision == FASTPI_MIXED, t))
        st = group_set_tuning(h->grp, t, h->stream);
    return st;
}

int fastpi_svd(fastpi_handle* h, const int64_t* rowptr, const int32_t* col, const double* val,
               double* U, double* S, double* V) {
    (void)rowptr;
    (void)col;
    if (!h || !h->inst.dp.valid) {
        set_error("no plan uploaded to this handle");
        return FASTPI_EINVAL;
    }
    const DevicePlan& d = h->inst.dp;
    if ((!val && d.nnz > 0) || (!U && d.m * d.r > 0) || (!S && d.r > 0) || (!V && d.n * d.r > 0)) {
        set_error("null device pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    return group_svd(h->grp, &val, &U, &S, &V, run_cfg(h, h->use_graph));
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
    const bool mixed = h->opts.precision == FASTPI_MIXED;
    const int sp = gemm_tn_splits(r, L, m, mixed, h->grp.ncu);
    const size_t need = static_cast<size_t>(r + r * L + static_cast<int64_t>(sp) * r * L) * sizeof(double);
    int rc = grow(h->aws, h->aws_bytes, need, st, "apply scratch");
    if (rc != FASTPI_OK) return rc;
    double* inv = h->aws;
    double* W = inv + r;
    double* part = W + r * L;
    launch_pinv_sigma(S, r, static_cast<double>(std::max(m, n)) * DBL_EPSILON, inv, st);
    launch_gemm_tn(U, r, Y, L, r, L, m, W, L, inv, nullptr, part, sp, st, mixed);
    launch_gemm_nn(V, r, nullptr, W, L, n, L, r, Z, L, nullptr, st, mixed);
    return check_launch();
}

}  // extern "C"

// Scratch of fastpi_apply_noalloc: one file-scope device array per GPU (the code object's
// copy on that device), resolved to a device address once per device with
// hipGetSymbolAddress; host code only ever uses that address, never the array's name.
constexpr int64_t kNoAllocApplyDoubles = int64_t(8) << 20;   // 64 MiB
static __device__ __align__(256) double scratch[kNoAllocApplyDoubles];
constexpr int kMaxDevices = 64;
static double* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// device address of this device's scratch (resolved on first use, with the device current)
static int noalloc_scratch(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("device index out of range for the no-allocation scratch");
        return FASTPI_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
            return FASTPI_EHIP;
        }
        g_scratch_ptr[device] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[device];
    return FASTPI_OK;
}

extern "C" {

int fastpi_apply_noalloc(fastpi_handle* h, int64_t m, int64_t n, int64_t r, const double* U,
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
    // the same split of U^T Y as fastpi_apply where it fits the scratch, fewer splits otherwise
    const int64_t rl = r * L;
    if (rl > (kNoAllocApplyDoubles - r) / 2) {
        set_error("fastpi_apply_noalloc: r * L = " + std::to_string(rl) + " needs more than the " +
                  std::to_string(kNoAllocApplyDoubles) + "-double scratch (at most r + 2 r L doubles)");
        return FASTPI_EINVAL;
    }
    const int64_t fit = (kNoAllocApplyDoubles - r - rl) / rl;
    const bool mixed = h->opts.precision == FASTPI_MIXED;
    const int sp = static_cast<int>(std::min<int64_t>(gemm_tn_splits(r, L, m, mixed, h->grp.ncu), fit));
    HIP_TRY(hipSetDevice(h->device));
    double* base = nullptr;
    int rc = noalloc_scratch(h->device, &base);
    if (rc != FASTPI_OK) return rc;
    hipStream_t st = h->stream;
    double* inv = base;
    double* W = inv + r;
    double* part = W + rl;
    launch_pinv_sigma(S, r, static_cast<double>(std::max(m, n)) * DBL_EPSILON, inv, st);
    launch_gemm_tn(U, r, Y, L, r, L, m, W, L, inv, nullptr, part, sp, st, mixed);
    launch_gemm_nn(V, r, nullptr, W, L, n, L, r, Z, L, nullptr, st, mixed);
    return check_launch();
}

int fastpi_labels_create(fastpi_labels** out, fastpi_handle* h, int64_t m, int64_t L,
                         const int64_t* rowptr, const int32_t* col, const double* val) {
    if (!out || !h || m < 0 || L < 0 || L > INT32_MAX || m > INT32_MAX || !rowptr) {
        set_error("bad labels arguments");
        return FASTPI_EINVAL;
    }
    *out = nullptr;
    if (rowptr[0] != 0) {
        set_error("label rowptr[0] must be 0");
        return FASTPI_EINVAL;
    }
    for (int64_t i = 0; i < m; ++i)
        if (rowptr[i + 1] < rowptr[i]) {
            set_error("label rowptr is not monotone at row " + std::to_string(i));
            return FASTPI_EINVAL;
        }
    const int64_t nnz = rowptr[m];
    if (nnz > 0 && !col) {
        set_error("null label column array");
        return FASTPI_EINVAL;
    }
    for (int64_t e = 0; e < nnz; ++e) {
        if (col[e] < 0 || col[e] >= L) {
            set_error("label index out of range at entry " + std::to_string(e));
            return FASTPI_EINVAL;
        }
        if (val && !std::isfinite(val[e])) {
            set_error("non-finite label value at entry " + std::to_string(e));
            return FASTPI_ENONFINITE;
        }
    }
    // transpose: per label, its rows in increasing order (counting sort is stable)
    std::vector<int64_t> lptr(static_cast<size_t>(L) + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) ++lptr[static_cast<size_t>(col[e]) + 1];
    for (int64_t l = 0; l < L; ++l) lptr[l + 1] += lptr[l];
    std::vector<int32_t> trow(static_cast<size_t>(nnz));
    std::vector<double> tval(static_cast<size_t>(nnz));
    std::vector<int64_t> fill(lptr.begin(), lptr.end() - 1);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int64_t d = fill[col[e]]++;
            trow[d] = static_cast<int32_t>(i);
            tval[d] = val ? val[e] : 1.0;
        }
    Segments sg;
    build_segments(lptr, sg);
    auto* y = new (std::nothrow) fastpi_labels();
    if (!y) {
        set_error("out of host memory");
        return FASTPI_ENOMEM;
    }
    y->device = h->device;
    y->m = m;
    y->L = L;
    y->nnz = nnz;
    auto fail = [&](int rc) {
        for (void* p : y->allocs) hipFree(p);
        delete y;
        return rc;
    };
    if (hipSetDevice(h->device) != hipSuccess) {
        set_error("hipSetDevice failed");
        return fail(FASTPI_EHIP);
    }
    if (nnz > 0) {
        void* p = nullptr;
        if (hipMalloc(&p, nnz * sizeof(int32_t)) != hipSuccess) {
            set_error("device allocation failed (labels)");
            return fail(FASTPI_ENOMEM);
        }
        y->allocs.push_back(p);
        y->rows = static_cast<int32_t*>(p);
        if (hipMalloc(&p, nnz * sizeof(double)) != hipSuccess) {
            set_error("device allocation failed (labels)");
            return fail(FASTPI_ENOMEM);
        }
        y->allocs.push_back(p);
        y->vals = static_cast<double*>(p);
        if (hipMemcpyAsync(y->rows, trow.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice, h->stream) !=
                hipSuccess ||
            hipMemcpyAsync(y->vals, tval.data(), nnz * sizeof(double), hipMemcpyHostToDevice, h->stream) !=
                hipSuccess) {
            set_error("label upload failed");
            return fail(FASTPI_EHIP);
        }
    }
    int rc = upload_segments(y->allocs, sg, y->seg, h->stream);
    if (rc != FASTPI_OK) return fail(rc);
    // the row-blocked form: labelled rows in blocks of at most kLabelBlockRows rows and
    // kLabelBlockPos positives, each block's positives by (sub-label, row), every block's
    // entries starting 16-byte aligned (padding entries are never addressed by a run)
    std::vector<int32_t> lrows, bstart;
    int64_t maxrow = 0;
    for (int64_t i = 0; i < m; ++i)
        if (rowptr[i + 1] > rowptr[i]) {
            lrows.push_back(static_cast<int32_t>(i));
            maxrow = std::max(maxrow, rowptr[i + 1] - rowptr[i]);
        }
    const int64_t nl = static_cast<int64_t>(lrows.size());
    bstart.push_back(0);
    for (int64_t k = 0, rows = 0, pos = 0; k < nl; ++k) {
        const int64_t d = rowptr[lrows[k] + 1] - rowptr[lrows[k]];
        if (rows == kLabelBlockRows || pos + d > kLabelBlockPos) {
            bstart.push_back(static_cast<int32_t>(k));
            rows = pos = 0;
        }
        ++rows;
        pos += d;
    }
    if (nl > 0) bstart.push_back(static_cast<int32_t>(nl));
    const int64_t nblk = static_cast<int64_t>(bstart.size()) - 1;
    std::vector<int32_t> bbase, rg, rv, re;   // block starts, group starts, runs (see LabelBlocks)
    std::vector<uint8_t> prow;
    std::vector<double> pval;
    bool ones = true;
    for (int64_t e = 0; e < nnz && val; ++e) ones = ones && val[e] == 1.0;
    // sub-labels: the thread slots the launch has beyond L go to the most frequent labels,
    // one at a time to the label with the most positives per sub-label
    std::vector<int64_t> lcount(static_cast<size_t>(L), 0);
    for (int64_t e = 0; e < nnz; ++e) ++lcount[col[e]];
    std::vector<int32_t> K(static_cast<size_t>(L), 1), vbase(static_cast<size_t>(L) + 1, 0);
    {
        int64_t spare = label_slots(L) - L;
        std::priority_queue<std::pair<double, int64_t>> heap;
        for (int64_t l = 0; l < L; ++l)
            if (lcount[l] > std::max<int64_t>(1, nblk)) heap.push({static_cast<double>(lcount[l]), l});
        while (spare > 0 && !heap.empty()) {
            const int64_t l = heap.top().second;
            heap.pop();
            ++K[l];
            --spare;
            const double per = static_cast<double>(lcount[l]) / K[l];
            if (per > static_cast<double>(std::max<int64_t>(1, nblk))) heap.push({per, l});
        }
    }
    for (int64_t l = 0; l < L; ++l) vbase[l + 1] = vbase[l] + K[l];
    const int64_t Lv = vbase[L];
    const int64_t padded = nnz + 16 * nblk;   // bound on the aligned layout's size
    const int64_t ngroup = label_groups(Lv);
    if (nnz > 0 && maxrow <= kLabelBlockPos && padded < INT32_MAX && nblk * (ngroup + 1) < INT32_MAX) {
        bbase.assign(static_cast<size_t>(nblk) + 1, 0);
        rg.assign(static_cast<size_t>(nblk * (ngroup + 1)), 0);
        prow.assign(static_cast<size_t>(padded), 0);
        if (!ones) pval.assign(static_cast<size_t>(padded), 0.0);
        int64_t base = 0;
        std::vector<int64_t> cnt(static_cast<size_t>(Lv) + 1), seen(static_cast<size_t>(L), 0);
        std::vector<int32_t> sub;   // sub-label of each of the block's positives, in row order
        for (int64_t b = 0; b < nblk; ++b) {
            const int64_t k0 = bstart[b], k1 = bstart[b + 1];
            bbase[b] = static_cast<int32_t>(base);
            // the i-th positive of label l in the block goes to sub-label vbase[l] + i mod K_l;
            // then a counting sort by sub-label (stable: rows stay increasing)
            sub.clear();
            for (int64_t k = k0; k < k1; ++k)
                for (int64_t e = rowptr[lrows[k]]; e < rowptr[lrows[k] + 1]; ++e) {
                    const int32_t l = col[e];
                    sub.push_back(vbase[l] + static_cast<int32_t>(seen[l]++ % K[l]));
                }
            for (int64_t k = k0; k < k1; ++k)
                for (int64_t e = rowptr[lrows[k]]; e < rowptr[lrows[k] + 1]; ++e) seen[col[e]] = 0;
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int32_t v : sub) ++cnt[v + 1];
            for (int64_t v = 0; v < Lv; ++v) cnt[v + 1] += cnt[v];
            // runs: one per sub-label present, in sub-label order, then the block's sentinel
            int64_t grp = 0;
            for (int64_t v = 0; v < Lv; ++v) {
                while (grp <= v / kLabelSubGroup && grp < ngroup)
                    rg[b * (ngroup + 1) + grp++] = static_cast<int32_t>(rv.size());
                if (cnt[v + 1] > cnt[v]) {
                    rv.push_back(static_cast<int32_t>(v));
                    re.push_back(static_cast<int32_t>(cnt[v]));
                }
            }
            while (grp <= ngroup) rg[b * (ngroup + 1) + grp++] = static_cast<int32_t>(rv.size());
            rv.push_back(-1);
            re.push_back(static_cast<int32_t>(cnt[Lv]));
            size_t q = 0;
            for (int64_t k = k0; k < k1; ++k)
                for (int64_t e = rowptr[lrows[k]]; e < rowptr[lrows[k] + 1]; ++e) {
                    const int64_t d = base + cnt[sub[q++]]++;
                    prow[d] = static_cast<uint8_t>(k - k0);
                    if (!ones) pval[d] = val[e];
                }
            base = (base + static_cast<int64_t>(sub.size()) + 15) / 16 * 16;
        }
        bbase[nblk] = static_cast<int32_t>(base);
        prow.resize(static_cast<size_t>(base));
        if (!ones) pval.resize(static_cast<size_t>(base));
        auto up = [&](const void* src, size_t bytes, void** dst) {
            if (hipMalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) {
                set_error("device allocation failed (label blocks)");
                return FASTPI_ENOMEM;
            }
            y->allocs.push_back(*dst);
            if (bytes > 0 && hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, h->stream) != hipSuccess) {
                set_error("label upload failed");
                return FASTPI_EHIP;
            }
            return FASTPI_OK;
        };
        void* d = nullptr;
        LabelBlocks& lb = y->lb;
        if ((rc = up(lrows.data(), lrows.size() * sizeof(int32_t), &d)) != FASTPI_OK) return fail(rc);
        lb.lrows = static_cast<int32_t*>(d);
        if ((rc = up(bstart.data(), bstart.size() * sizeof(int32_t), &d)) != FASTPI_OK) return fail(rc);
        lb.bstart = static_cast<int32_t*>(d);
        if ((rc = up(vbase.data(), vbase.size() * sizeof(int32_t), &d)) != FASTPI_OK) return fail(rc);
        lb.vbase = static_cast<int32_t*>(d);
        if ((rc = up(bbase.data(), bbase.size() * sizeof(int32_t), &d)) != FASTPI_OK) return fail(rc);
        lb.bbase = static_cast<int32_t*>(d);
        if ((rc = up(rg.data(), rg.size() * sizeof(int32_t), &d)) != FASTPI_OK) return fail(rc);
        lb.rg = static_cast<int32_t*>(d);
        if ((rc = up(rv.data(), rv.size() * sizeof(int32_t), &d)) != FASTPI_OK) return fail(rc);
        lb.rv = static_cast<int32_t*>(d);
        if ((rc = up(re.data(), re.size() * sizeof(int32_t), &d)) != FASTPI_OK) return fail(rc);
        lb.re = static_cast<int32_t*>(d);
        if ((rc = up(prow.data(), prow.size(), &d)) != FASTPI_OK) return fail(rc);
        lb.prow = static_cast<uint8_t*>(d);
        if (!ones) {
            if ((rc = up(pval.data(), pval.size() * sizeof(double), &d)) != FASTPI_OK) return fail(rc);
            lb.pval = static_cast<double*>(d);
        }
        lb.nblk = nblk;
        lb.Lv = Lv;
        y->blocked = true;
    }
    // the host tables above go out of scope: wait for the copies
    if (hipStreamSynchronize(h->stream) != hipSuccess) {
        set_error("label upload failed");
        return fail(FASTPI_EHIP);
    }
    *out = y;
    return FASTPI_OK;
}

void fastpi_labels_destroy(fastpi_labels* y) {
    if (!y) return;
    hipSetDevice(y->device);
    hipDeviceSynchronize();
    for (void* p : y->allocs) hipFree(p);
    delete y;
}

int fastpi_labels_nnz(const fastpi_labels* y, int64_t* nnz) {
    if (!y || !nnz) {
        set_error("null labels or output");
        return FASTPI_EINVAL;
    }
    *nnz = y->nnz;
    return FASTPI_OK;
}

int fastpi_apply_sparse(fastpi_handle* h, int64_t m, int64_t n, int64_t r, const double* U,
                        const double* S, const double* V, const fastpi_labels* Y, double* Z) {
    if (!h || !Y || m <= 0 || n <= 0 || r < 0 || Y->m != m || Y->device != h->device) {
        set_error("bad handle, labels or sizes (the labels must have m rows, on the handle's device)");
        return FASTPI_EINVAL;
    }
    const int64_t L = Y->L;
    if (L == 0) return FASTPI_OK;
    if (!Z || (r > 0 && (!U || !S || !V))) {
        set_error("null device pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    hipStream_t st = h->stream;
    if (r == 0) {
        launch_fill(Z, n * L, 0.0, st);
        return check_launch();
    }
    const int64_t npart = Y->blocked ? label_spmm_chunks(Y->lb.nblk, r, Y->lb.Lv) * Y->lb.Lv : Y->seg.npart;
    const size_t need = static_cast<size_t>(r + L * r + npart * r) * sizeof(double);
    int rc = grow(h->aws, h->aws_bytes, need, st, "apply scratch");
    if (rc != FASTPI_OK) return rc;
    double* inv = h->aws;
    double* C = inv + r;          // L x r: Y^T U diag(S^+)
    double* part = C + L * r;
    launch_pinv_sigma(S, r, static_cast<double>(std::max(m, n)) * DBL_EPSILON, inv, st);
    if (Y->blocked) {
        launch_label_spmm(Y->lb, U, r, L, inv, C, part, st, &h->timer);
    } else {
        launch_fill(C, L * r, 0.0, st);   // labels without a positive keep a zero row
        launch_spmm_rows(Y->seg, Y->rows, Y->vals, U, r, inv, C, r, nullptr, false, part, st, &h->timer);
    }
    launch_gemm_nt(V, r, C, r, n, L, r, Z, L, st, h->opts.precision == FASTPI_MIXED, &h->timer);
    return check_launch();
}

int fastpi_topk_hits(fastpi_handle* h, int64_t rows, int64_t n, int64_t L, const int64_t* rowptr,
                     const int32_t* col, const double* val, const double* Z, const int64_t* y_rowptr,
                     const int32_t* y_col, int32_t nk, const int32_t* ks, int32_t* hits) {
    if (!h || rows < 0 || n < 0 || L < 0 || L > INT32_MAX - 1 || nk < 1 || nk > kTopkMaxKs || !ks) {
        set_error("bad handle or sizes (1 <= nk <= 16)");
        return FASTPI_EINVAL;
    }
    int kmax = 0;
    for (int i = 0; i < nk; ++i) {
        if (ks[i] < 1 || ks[i] > kTopkMaxK) {
            set_error("every k must lie in [1, 64]");
            return FASTPI_EINVAL;
        }
        kmax = std::max(kmax, static_cast<int>(ks[i]));
    }
    if (rows == 0) return FASTPI_OK;
    if (!rowptr || !col || !val || !Z || !y_rowptr || !y_col || !hits) {
        set_error("null device pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    const int64_t sd = topk_scratch_doubles(rows, L);
    if (sd > 0) {
        int rc = grow(h->ews, h->ews_bytes, static_cast<size_t>(sd) * sizeof(double), h->stream, "evaluation scratch");
        if (rc != FASTPI_OK) return rc;
    }
    launch_topk_hits(rows, n, L, rowptr, col, val, Z, y_rowptr, y_col, nk, ks, kmax, hits, h->ews, h->stream,
                     &h->timer);
    return check_launch();
}

int fastpi_stage_output(fastpi_handle* h, int which, double* dst, int64_t count) {
    if (!h || !h->inst.dp.valid || !dst) {
        set_error("bad handle or pointer");
        return FASTPI_EINVAL;
    }
    const Instance& I = h->inst;
    const DevicePlan& d = I.dp;
    const double* src = nullptr;
    int64_t want = 0;
    switch (which) {
        case 0: src = I.ws + I.o_sig1; want = d.s_b; break;
        case 1: src = I.ws + I.o_sig2; want = d.s; break;
        case 2: src = I.ws + I.o_v2; want = d.n1 * d.s; break;
        case 3: src = I.ws + I.o_u2; want = d.m * d.s; break;
        default: set_error("unknown stage"); return FASTPI_EINVAL;
    }
    if (count != want) {
        set_error("stage size mismatch: expected " + std::to_string(want));
        return FASTPI_EINVAL;
    }
    if (want > 0) launch_copy(src, want, dst, h->stream);
    return check_launch();
}

int fastpi_syev_top(fastpi_handle* h, int64_t q, const double* G, int64_t t, double* vals,
                    double* vecs) {
    if (!h || q <= 0 || t <= 0 || t > q || !G || !vals || !vecs) {
        set_error("bad arguments");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    const int rows = h->grp.tune.gram_rows;
    int st = grow(h->sws, h->sws_bytes, eig_job_doubles(q, rows) * sizeof(double), h->stream, "eigensolver");
    if (st != FASTPI_OK) return st;
    if ((st = grow(h->siws, h->siws_bytes, eig_job_ints(q) * sizeof(int), h->stream, "eigensolver")) != FASTPI_OK)
        return st;
    const bool precond = h->grp.tune.precond != 0;
    if (precond &&
        (st = grow(h->sa, h->sa_bytes, static_cast<size_t>(q * q) * sizeof(double), h->stream, "eigensolver")) !=
            FASTPI_OK)
        return st;
    EigSet es;
    std::vector<EigJob> jobs{eig_make_job(G, precond ? h->sa : nullptr, q, t, vals, vecs, h->sws, h->siws, nullptr,
                                          h->opts.tol, rows, 0)};
    if ((st = eig_set_create(es, jobs, rows, precond, h->grp.tune.eig_fused != 0, h->stream)) != FASTPI_OK) {
        eig_set_free(es);
        set_error("eigensolver allocation failed");
        return st;
    }
    eig_begin(es, h->stream);
    st = eig_iterate(es, h->opts.max_sweeps, h->grp.tune.inner_sweeps, h->stream, h->copy_stream, &h->timer,
                     nullptr);
    if (st == FASTPI_OK) {
        eig_end(es, h->stream);
        if (hipStreamSynchronize(h->stream) != hipSuccess) st = FASTPI_EHIP;
    }
    h->syev_sweeps = es.host_state[kEigStSweeps];
    const bool capped = es.host_state[kEigStCapped] != 0;
    eig_set_free(es);
    if (st != FASTPI_OK) return st;
    if (capped) {
        set_error("eigensolver reached the sweep cap");
        return FASTPI_ENOCONV;
    }
    return check_launch();
}

int fastpi_mfma_gemm(fastpi_handle* h, int ta, int tb, int64_t M, int64_t N, int64_t K, const double* A,
                     int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc, int fp32) {
    if (!h || M < 0 || N < 0 || K < 0 || (M * N > 0 && (!C || ldc < N)) ||
        (M * N * K > 0 && (!A || !B || lda < (ta ? M : K) || ldb < (tb ? K : N)))) {
        set_error("bad handle, shape, leading dimension or pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    launch_mfma_gemm(ta != 0, tb != 0, A, lda, B, ldb, M, N, K, C, ldc, 1, 0, h->stream, fp32 != 0);
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
    h->inst.sweeps[0] = h->host_pinned[1];
    return decode_status(h->host_pinned[0]);
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

static bool rank_model_valid(const fastpi_rank_model* m) {
    if (!m || !m->mean || !m->std || !m->lo || !m->hi || !(m->margin >= 0.0)) return false;
    for (int j = 0; j < kRankFeatures; ++j)
        if (!(m->std[j] > 0.0)) return false;
    return true;
}

int fastpi_rank_inputs(int64_t n, const double* feats, const fastpi_rank_model* model, float* X,
                       int32_t* in_range) {
    if (n < 0 || (n > 0 && !feats) || !rank_model_valid(model)) {
        set_error("bad arguments (null pointer, n < 0, std <= 0 or negative margin)");
        return FASTPI_EINVAL;
    }
    rank_inputs(n, feats, *model, X, in_range);
    return FASTPI_OK;
}

int fastpi_rank_allocate(int64_t n, const float* f, const int64_t* q, int64_t budget, int64_t* s) {
    if (n < 0 || (n > 0 && (!f || !q || !s))) {
        set_error("bad arguments");
        return FASTPI_EINVAL;
    }
    for (int64_t i = 0; i < n; ++i)
        if (q[i] < 0) {
            set_error("negative block capacity");
            return FASTPI_EINVAL;
        }
    rank_allocate(n, f, q, budget, s);
    return FASTPI_OK;
}

int fastpi_plan_learned_ranks(const fastpi_plan* plan, fastpi_handle* h, const double* val,
                              const fastpi_rank_model* model, const float* theta, int64_t* ranks) {
    if (!plan || !h || !val || !theta || !ranks || !rank_model_valid(model)) {
        set_error("bad arguments (null pointer, std <= 0 or negative margin)");
        return FASTPI_EINVAL;
    }
    const Plan& P = plan->p;
    const std::vector<BlockDesc>& blocks = P.ro.blocks;
    const int64_t B = static_cast<int64_t>(blocks.size());
    std::vector<int64_t> dense;   // block ids of the dense blocks, in block order
    for (int64_t b = 0; b < B; ++b)
        if (blocks[b].rows > 0 && blocks[b].cols > 0) dense.push_back(b);
    const int64_t nd = static_cast<int64_t>(dense.size());
    std::vector<double> feats(static_cast<size_t>(nd) * kRankFeatures);
    if (nd > 0) {
        const int rc = block_features(P, val, feats.data());
        if (rc != FASTPI_OK) return rc;
    }
    std::vector<float> X(static_cast<size_t>(nd) * kRankFeatures);
    std::vector<int32_t> ok(nd);
    rank_inputs(nd, feats.data(), *model, X.data(), ok.data());
    // the alpha rule: the fallback of out-of-range blocks and the total budget
    std::vector<int64_t> alpha_rank(nd), q(nd);
    int64_t budget = 0, kept = 0, nin = 0;
    for (int64_t i = 0; i < nd; ++i) {
        const BlockDesc& d = blocks[dense[i]];
        q[i] = std::min(d.rows, d.cols);
        alpha_rank[i] = std::min({target_rank(P.alpha, d.cols), d.rows, d.cols});
        budget += alpha_rank[i];
        if (ok[i]) ++nin;
        else kept += alpha_rank[i];
    }
    std::vector<int64_t> out(nd);
    for (int64_t i = 0; i < nd; ++i) out[i] = alpha_rank[i];
    if (nin > 0) {
        std::vector<float> Xin(static_cast<size_t>(nin) * kRankFeatures), f(nin);
        std::vector<int64_t> qin(nin), s_in(nin);
        for (int64_t i = 0, k = 0; i < nd; ++i)
            if (ok[i]) {
                std::copy(X.begin() + i * kRankFeatures, X.begin() + (i + 1) * kRankFeatures,
                          Xin.begin() + k * kRankFeatures);
                qin[k++] = q[i];
            }
        HIP_TRY(hipSetDevice(h->device));
        void* dX = nullptr;
        void* df = nullptr;
        if (hipMalloc(&dX, Xin.size() * sizeof(float)) != hipSuccess ||
            hipMalloc(&df, f.size() * sizeof(float)) != hipSuccess) {
            if (dX) hipFree(dX);
            set_error("device allocation failed (rank-network input)");
            return FASTPI_ENOMEM;
        }
        hipError_t e = hipMemcpyAsync(dX, Xin.data(), Xin.size() * sizeof(float), hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) {
            launch_mlp_forward(nin, static_cast<const float*>(dX), theta, static_cast<float*>(df), nullptr, h->stream);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(f.data(), df, f.size() * sizeof(float), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        hipFree(dX);
        hipFree(df);
        if (e != hipSuccess) {
            set_error(std::string("HIP error in the rank network: ") + hipGetErrorString(e));
            return FASTPI_EHIP;
        }
        rank_allocate(nin, f.data(), qin.data(), budget - kept, s_in.data());
        for (int64_t i = 0, k = 0; i < nd; ++i)
            if (ok[i]) out[i] = s_in[k++];
    }
    std::fill(ranks, ranks + B, 0);
    for (int64_t i = 0; i < nd; ++i) ranks[dense[i]] = out[i];
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
    if (!h || kind < KT_NONE || kind > KT_LAST) {
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
    for (int i = 0; i < 3; ++i) out3[i] = h->inst.sweeps[i];
    if (!h->inst.dp.valid) out3[1] = h->syev_sweeps;
    return st;
}

int fastpi_last_rotations(fastpi_handle* h, int64_t* out2) {
    if (!h || !out2) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    out2[0] = h->inst.rotated[0];
    out2[1] = h->inst.rotated[1];
    return FASTPI_OK;
}

int fastpi_set_graph(fastpi_handle* h, int enable) {
    if (!h) {
        set_error("null handle");
        return FASTPI_EINVAL;
    }
    h->use_graph = enable != 0;
    return FASTPI_OK;
}

int64_t fastpi_last_graph_launches(const fastpi_handle* h) { return h ? h->grp.graph_launches : -1; }

int fastpi_set_tuning(fastpi_handle* h, const fastpi_tuning* t) {
    if (!h || !t) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    return group_set_tuning(h->grp, from_c(*t), h->stream);
}

int fastpi_get_tuning(const fastpi_handle* h, fastpi_tuning* t) {
    if (!h || !t) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    to_c(h->grp.tune, t);
    return FASTPI_OK;
}

static InnerCfg inner_from_c(const fastpi_inner& c) {
    InnerCfg o;
    o.mode = c.mode;
    o.oversample = c.oversample;
    o.iters = c.iters;
    o.seed = c.seed;
    return o;
}

static void inner_to_c(const InnerCfg& c, fastpi_inner* o) {
    o->mode = c.mode;
    o->oversample = c.oversample;
    o->iters = c.iters;
    o->seed = c.seed;
}

int fastpi_set_block_route(fastpi_handle* h, double min_cost) {
    if (!h || !(min_cost >= 0)) {
        set_error("bad handle or cost");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    h->grp.big_cost = min_cost;
    if (!h->inst.dp.valid) return FASTPI_OK;
    HIP_TRY(hipStreamSynchronize(h->stream));
    return group_build(h->grp, h->device, h->stream);
}

int fastpi_batch_set_block_route(fastpi_batch* b, double min_cost) {
    if (!batch_live(b)) return FASTPI_EINVAL;
    if (!b || !(min_cost >= 0)) {
        set_error("bad batch or cost");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(b->h->device));
    b->grp.big_cost = min_cost;
    HIP_TRY(hipStreamSynchronize(b->h->stream));
    return group_build(b->grp, b->h->device, b->h->stream);
}

int fastpi_set_inner(fastpi_handle* h, const fastpi_inner* c) {
    if (!h || !c) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    return group_set_inner(h->grp, inner_from_c(*c), h->stream);
}

int fastpi_get_inner(const fastpi_handle* h, fastpi_inner* c) {
    if (!h || !c) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    inner_to_c(h->grp.inner, c);
    return FASTPI_OK;
}

}  // extern "C"

static CoreCfg core_from_c(const fastpi_core_solver& c) {
    CoreCfg o;
    o.mode = c.mode;
    o.min_order = c.min_order;
    o.k_factor = c.k_factor;
    o.max_frac = c.max_frac;
    o.iters_fp64 = c.iters_fp64;
    o.iters_mixed = c.iters_mixed;
    o.orth_every = c.orth_every;
    o.res_tol_fp64 = c.res_tol_fp64;
    o.res_tol_mixed = c.res_tol_mixed;
    o.k_factor_mixed = c.k_factor_mixed;
    return o;
}

extern "C" {

int fastpi_set_core_solver(fastpi_handle* h, const fastpi_core_solver* c) {
    if (!h || !c) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    return group_set_core(h->grp, core_from_c(*c), h->stream);
}

int fastpi_get_core_solver(const fastpi_handle* h, fastpi_core_solver* c) {
    if (!h || !c) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    const CoreCfg& o = h->grp.core;
    *c = fastpi_core_solver{};
    c->mode = o.mode;
    c->min_order = o.min_order;
    c->k_factor = o.k_factor;
    c->max_frac = o.max_frac;
    c->iters_fp64 = o.iters_fp64;
    c->iters_mixed = o.iters_mixed;
    c->orth_every = o.orth_every;
    c->res_tol_fp64 = o.res_tol_fp64;
    c->res_tol_mixed = o.res_tol_mixed;
    c->k_factor_mixed = o.k_factor_mixed;
    return FASTPI_OK;
}

int fastpi_batch_set_core_solver(fastpi_batch* b, const fastpi_core_solver* c) {
    if (!batch_live(b)) return FASTPI_EINVAL;
    if (!c) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(b->h->device));
    return group_set_core(b->grp, core_from_c(*c), b->h->stream);
}

int fastpi_last_core_routes(const fastpi_handle* h, int32_t* out2) {
    if (!h || !out2) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    out2[0] = h->inst.route[0];
    out2[1] = h->inst.route[1];
    return FASTPI_OK;
}

int fastpi_batch_core_routes(const fastpi_batch* b, int32_t* out) {
    if (!b || !out) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    for (size_t i = 0; i < b->inst.size(); ++i) {
        out[2 * i] = b->inst[i].route[0];
        out[2 * i + 1] = b->inst[i].route[1];
    }
    return FASTPI_OK;
}

int fastpi_gaussian(fastpi_handle* h, int64_t count, uint32_t seed, uint32_t stream, double* out) {
    if (!h || count < 0 || (count > 0 && !out)) {
        set_error("bad handle, count or pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    launch_gauss(out, count, seed, stream, h->stream);
    return check_launch();
}

int fastpi_inner_applies(const fastpi_inner* c, int64_t t, int64_t q) {
    if (!c) return 0;
    return inner_applies(inner_from_c(*c), t, q) ? 1 : 0;
}

int fastpi_set_tuning_cache(fastpi_handle* h, const char* path) {
    if (!h) {
        set_error("null handle");
        return FASTPI_EINVAL;
    }
    h->tune_cache = path ? path : "";
    return FASTPI_OK;
}

int fastpi_autotune(fastpi_handle* h, const double* val, double* U, double* S, double* V,
                    char* report, int64_t report_cap) {
    if (!h || !h->inst.dp.valid) {
        set_error("no plan uploaded to this handle");
        return FASTPI_EINVAL;
    }
    const DevicePlan& d = h->inst.dp;
    if ((!val && d.nnz > 0) || (!U && d.m * d.r > 0) || (!S && d.r > 0) || (!V && d.n * d.r > 0)) {
        set_error("null device pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(h->device));
    std::string rep;
    const int st = group_autotune(h->grp, &val, &U, &S, &V, run_cfg(h, false),
                                  h->tune_cache.empty() ? nullptr : h->tune_cache.c_str(), h->device, &rep);
    copy_report(rep, report, report_cap);
    return st;
}

// ---------------------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------------------
int fastpi_batch_create(fastpi_batch** b, fastpi_handle* h, int64_t count,
                        const fastpi_plan* const* plans) {
    if (!b || !h || count <= 0 || !plans) {
        set_error("bad arguments");
        return FASTPI_EINVAL;
    }
    *b = nullptr;
    for (int64_t i = 0; i < count; ++i)
        if (!plans[i]) {
            set_error("null plan in the batch");
            return FASTPI_EINVAL;
        }
    HIP_TRY(hipSetDevice(h->device));
    fastpi_batch* B = new (std::nothrow) fastpi_batch();
    if (!B) {
        set_error("host allocation failed");
        return FASTPI_ENOMEM;
    }
    B->h = h;
    h->batches.push_back(B);
    B->inst.resize(static_cast<size_t>(count));
    void* p = nullptr;
    const size_t words = static_cast<size_t>(2 * count + 16);
    if (hipMalloc(&p, words * sizeof(int)) != hipSuccess) {
        fastpi_batch_destroy(B);
        set_error("device allocation failed (batch status)");
        return FASTPI_ENOMEM;
    }
    B->status = static_cast<int*>(p);
    if (hipHostMalloc(&p, words * sizeof(int), hipHostMallocDefault) != hipSuccess) {
        fastpi_batch_destroy(B);
        set_error("pinned host allocation failed");
        return FASTPI_ENOMEM;
    }
    B->host_status = static_cast<int*>(p);
    launch_fill_i32(B->status, static_cast<int64_t>(words), 0, h->stream);
    int st = FASTPI_OK;
    for (int64_t i = 0; i < count && st == FASTPI_OK; ++i) {
        B->inst[i].status = B->status + 2 * i;
        st = instance_upload(B->inst[i], plans[i]->p, h->opts.max_workspace_bytes, h->stream);
    }
    if (st == FASTPI_OK) {
        for (Instance& I : B->inst) B->grp.inst.push_back(&I);
        B->grp.inner = h->grp.inner;
        B->grp.core = h->grp.core;
        B->grp.big_cost = h->grp.big_cost;
        B->grp.eig_tol = h->grp.eig_tol;
        B->grp.mixed = h->opts.precision == FASTPI_MIXED;
        st = group_build(B->grp, h->device, h->stream);
    }
    Tuning t;
    if (st == FASTPI_OK && !h->tune_cache.empty() &&
        tuning_lookup(B->grp, h->tune_cache.c_str(), h->device, h->opts.precision == FASTPI_MIXED, t))
        st = group_set_tuning(B->grp, t, h->stream);
    if (st != FASTPI_OK) {
        fastpi_batch_destroy(B);
        return st;
    }
    *b = B;
    return check_launch();
}

// frees a batch's device resources on its handle's device and stream (handle alive)
static void batch_release(fastpi_batch* b) {
    fastpi_handle* h = b->h;
    hipSetDevice(h->device);
    hipStreamSynchronize(h->stream);
    group_free(b->grp);
    for (Instance& I : b->inst) instance_free(I, h->stream);
    if (b->status) hipFree(b->status);
    if (b->host_status) hipHostFree(b->host_status);
    b->status = nullptr;
    b->host_status = nullptr;
}

void fastpi_batch_destroy(fastpi_batch* b) {
    if (!b) return;
    if (fastpi_handle* h = b->h) {
        batch_release(b);
        auto& v = h->batches;
        v.erase(std::remove(v.begin(), v.end(), b), v.end());
    }
    delete b;
}

// a batch whose handle is still alive
static bool batch_live(const fastpi_batch* b) {
    if (!b) {
        set_error("null batch");
        return false;
    }
    if (!b->h) {
        set_error("the batch's handle was destroyed");
        return false;
    }
    return true;
}

int fastpi_batch_svd(fastpi_batch* b, const double* const* val, double* const* U, double* const* S,
                     double* const* V) {
    if (!batch_live(b)) return FASTPI_EINVAL;
    if (!b || !val || !U || !S || !V) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    for (size_t i = 0; i < b->inst.size(); ++i) {
        const DevicePlan& d = b->inst[i].dp;
        if ((!val[i] && d.nnz > 0) || (!U[i] && d.m * d.r > 0) || (!S[i] && d.r > 0) || (!V[i] && d.n * d.r > 0)) {
            set_error("null device pointer for instance " + std::to_string(i));
            return FASTPI_EINVAL;
        }
    }
    HIP_TRY(hipSetDevice(b->h->device));
    return group_svd(b->grp, val, U, S, V, run_cfg(b->h, b->use_graph));
}

int fastpi_batch_sync(fastpi_batch* b, int32_t* status, int32_t* sweeps) {
    if (!batch_live(b)) return FASTPI_EINVAL;
    if (!b) {
        set_error("null batch");
        return FASTPI_EINVAL;
    }
    fastpi_handle* h = b->h;
    HIP_TRY(hipSetDevice(h->device));
    const size_t n = b->inst.size();
    HIP_TRY(hipMemcpyAsync(b->host_status, b->status, 2 * n * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    int first = FASTPI_OK;
    std::string first_msg;
    for (size_t i = 0; i < n; ++i) {
        b->inst[i].sweeps[0] = b->host_status[2 * i + 1];
        const int code = decode_status(b->host_status[2 * i]);
        if (status) status[i] = code;
        if (sweeps)
            for (int k = 0; k < 3; ++k) sweeps[3 * i + k] = b->inst[i].sweeps[k];
        // the first error wins over any warning
        if (code != FASTPI_OK && (first == FASTPI_OK || (first > 0 && code < 0))) {
            first = code;
            first_msg = "instance " + std::to_string(i) + ": " + fastpi_last_error();
        }
    }
    if (first != FASTPI_OK) set_error(first_msg);
    return first;
}

int fastpi_batch_rotations(const fastpi_batch* b, int64_t* out) {
    if (!b || !out) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    for (size_t i = 0; i < b->inst.size(); ++i) {
        out[2 * i] = b->inst[i].rotated[0];
        out[2 * i + 1] = b->inst[i].rotated[1];
    }
    return FASTPI_OK;
}

int fastpi_batch_set_graph(fastpi_batch* b, int enable) {
    if (!batch_live(b)) return FASTPI_EINVAL;
    if (!b) {
        set_error("null batch");
        return FASTPI_EINVAL;
    }
    b->use_graph = enable != 0;
    return FASTPI_OK;
}

int64_t fastpi_batch_last_graph_launches(const fastpi_batch* b) { return b ? b->grp.graph_launches : -1; }

int fastpi_batch_set_tuning(fastpi_batch* b, const fastpi_tuning* t) {
    if (!batch_live(b)) return FASTPI_EINVAL;
    if (!b || !t) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(b->h->device));
    return group_set_tuning(b->grp, from_c(*t), b->h->stream);
}

int fastpi_batch_set_inner(fastpi_batch* b, const fastpi_inner* c) {
    if (!batch_live(b)) return FASTPI_EINVAL;
    if (!b || !c) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    HIP_TRY(hipSetDevice(b->h->device));
    return group_set_inner(b->grp, inner_from_c(*c), b->h->stream);
}

int fastpi_batch_get_tuning(const fastpi_batch* b, fastpi_tuning* t) {
    if (!b || !t) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    to_c(b->grp.tune, t);
    return FASTPI_OK;
}

int fastpi_batch_autotune(fastpi_batch* b, const double* const* val, double* const* U, double* const* S,
                          double* const* V, char* report, int64_t report_cap) {
    if (!batch_live(b)) return FASTPI_EINVAL;
    if (!b || !val || !U || !S || !V) {
        set_error("null pointer");
        return FASTPI_EINVAL;
    }
    fastpi_handle* h = b->h;
    HIP_TRY(hipSetDevice(h->device));
    std::string rep;
    const int st = group_autotune(b->grp, val, U, S, V, run_cfg(h, false),
                                  h->tune_cache.empty() ? nullptr : h->tune_cache.c_str(), h->device, &rep);
    copy_report(rep, report, report_cap);
    return st;
}

}  // extern "C"
