// Value gather (split of the reordered matrix, Section 3.3) and the batched SVD of the
// diagonal blocks of A11 (Eq. 1) by one-sided (Hestenes) Jacobi, one workgroup per block.
#include <cfloat>

#include "device_common.h"
#include "kernels.h"

namespace fastpi {

// ---------------------------------------------------------------------------------------
// Gather: caller CSR values -> [dense A11 blocks | A21 CSR | A21 CSC | T CSR | T CSC].
// The destination indices come from the planner; the dense block region must be zero.
// Non-finite values raise bit 0 of *status.
// ---------------------------------------------------------------------------------------
__global__ void k_gather_values(const double* __restrict__ val, const int64_t* __restrict__ dst0,
                                const int64_t* __restrict__ dst1, int64_t nnz,
                                double* __restrict__ out, int* __restrict__ status) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < nnz;
         e += stride) {
        const double v = val[e];
        if (!isfinite(v)) atomicOr(status, 1);
        const int64_t d0 = dst0[e];
        if (d0 >= 0) out[d0] = v;
        const int64_t d1 = dst1[e];
        if (d1 >= 0) out[d1] = v;
    }
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = v;
}

void launch_fill(double* p, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return;
    const int blocks = static_cast<int>(std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_fill<double>, dim3(blocks), dim3(256), 0, st, p, n, v);
}
void launch_fill_i32(int* p, int64_t n, int v, hipStream_t st) {
    if (n <= 0) return;
    const int blocks = static_cast<int>(std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_fill<int>, dim3(blocks), dim3(256), 0, st, p, n, v);
}

void launch_gather(const double* val, const int64_t* dst0, const int64_t* dst1, int64_t nnz,
                   double* out, int* status, hipStream_t st) {
    if (nnz <= 0) return;
    const int blocks = static_cast<int>(std::min<int64_t>((nnz + 255) / 256, 8192));
    hipLaunchKernelGGL(k_gather_values, dim3(blocks), dim3(256), 0, st, val, dst0, dst1, nnz,
                       out, status);
}

// ---------------------------------------------------------------------------------------
// Batched one-sided Jacobi.
//
// Block i (rows x cols, column-major) is taken as X = A_i when rows >= cols and X = A_i^T
// otherwise, so X is p x q with p >= q. Column pairs of X are rotated until every pair is
// orthogonal to `tol` in the cosine sense; the rotations accumulate in J (q x q). Then
// X = W with orthogonal columns, W_c = sigma_c u_c, and A_i = U Sigma V^T with U = W Sigma^-1,
// V = J (or U = J, V = W Sigma^-1 for the transposed case). The s_i largest are kept,
// descending, ties to the lower column.
//
// Pairs follow the circle-method round robin: qe-1 rounds of qe/2 disjoint pairs per sweep
// (qe = q rounded up to even), each wave of the workgroup taking every NW-th pair.
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ void jacobi_sweeps(T* X, T* J, int p, int q, int max_sweeps, T tol,
                              int* sweeps_used, int* status) {
    constexpr int NT = 256;
    constexpr int NW = NT / kWave;
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    __shared__ int s_rot;
    const int qe = q + (q & 1);
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        if (threadIdx.x == 0) s_rot = 0;
        __syncthreads();
        int rotated = 0;
        for (int round = 0; round < qe - 1; ++round) {
            for (int pr = wave; pr < qe / 2; pr += NW) {
                int a, b;
                round_robin_pair(round, pr, qe, a, b);
                if (b >= q) continue;
                T* xa = X + static_cast<int64_t>(a) * p;
                T* xb = X + static_cast<int64_t>(b) * p;
                T al = 0, be = 0, ga = 0;
                for (int r = lane; r < p; r += kWave) {
                    const T u = xa[r], v = xb[r];
                    al += u * u;
                    be += v * v;
                    ga += u * v;
                }
                al = wave_sum(al);
                be = wave_sum(be);
                ga = wave_sum(ga);
                const T aga = ga < T(0) ? -ga : ga;
                if (!(al > T(0) && be > T(0)) || !(aga > tol * sqrt(al) * sqrt(be))) continue;
                T c, s, t;
                jacobi_rotation(al, be, ga, c, s, t);
                for (int r = lane; r < p; r += kWave) {
                    const T u = xa[r], v = xb[r];
                    xa[r] = c * u - s * v;
                    xb[r] = s * u + c * v;
                }
                T* ja = J + static_cast<int64_t>(a) * q;
                T* jb = J + static_cast<int64_t>(b) * q;
                for (int r = lane; r < q; r += kWave) {
                    const T u = ja[r], v = jb[r];
                    ja[r] = c * u - s * v;
                    jb[r] = s * u + c * v;
                }
                rotated = 1;
            }
            __syncthreads();
        }
        if (rotated) s_rot = 1;   // benign race: every writer stores 1
        __syncthreads();
        if (s_rot == 0) break;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(sweeps_used, sweep + 1);
        if (sweep == max_sweeps) atomicOr(status, 2);
    }
}

template <typename T>
__device__ void block_svd_one(const BlockTask& w, T* X, T* J, int max_sweeps, T tol) {
    const int rows = w.rows, cols = w.cols;
    const bool trans = rows < cols;
    const int p = trans ? cols : rows;
    const int q = trans ? rows : cols;
    const double* A = w.A;
    // X (p x q, column-major) and J = I
    for (int64_t e = threadIdx.x; e < static_cast<int64_t>(p) * q; e += blockDim.x) {
        const int r = static_cast<int>(e % p), c = static_cast<int>(e / p);
        const double v = trans ? A[static_cast<int64_t>(r) * rows + c] : A[static_cast<int64_t>(c) * rows + r];
        X[e] = static_cast<T>(v);
    }
    for (int e = threadIdx.x; e < q * q; e += blockDim.x) J[e] = (e % q == e / q) ? T(1) : T(0);
    __syncthreads();
    if (q > 1) jacobi_sweeps<T>(X, J, p, q, max_sweeps, tol, w.status + 1, w.status);
    __syncthreads();

    // column norms, then the descending rank of every column (ties: lower column first);
    // in LDS up to 256 columns, else in the block's global scratch after J (the same
    // workgroup writes and reads them, ordered by its barriers)
    __shared__ double l_sig[256];
    __shared__ int l_rank[256];
    double* s_sig = l_sig;
    int* s_rank = l_rank;
    if (q > 256) {
        s_sig = static_cast<double*>(w.scratch) + static_cast<int64_t>(p) * q + static_cast<int64_t>(q) * q;
        s_rank = reinterpret_cast<int*>(s_sig + q);
    }
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    for (int c = wave; c < q; c += blockDim.x / kWave) {
        double acc = 0;
        const T* xc = X + static_cast<int64_t>(c) * p;
        for (int r = lane; r < p; r += kWave) {
            const double v = static_cast<double>(xc[r]);
            acc += v * v;
        }
        acc = wave_sum(acc);
        if (lane == 0) s_sig[c] = isfinite(acc) ? sqrt(acc) : 0.0;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < q; c += blockDim.x) {
        int rk = 0;
        const double sc = s_sig[c];
        for (int d = 0; d < q; ++d) {
            const double sd = s_sig[d];
            rk += (sd > sc) || (sd == sc && d < c);
        }
        s_rank[c] = rk;
    }
    __syncthreads();
    const int si = w.rank;
    for (int c = 0; c < q; ++c) {
        const int k = s_rank[c];
        if (k >= si) continue;
        const double sc = s_sig[c];
        const double inv = sc > 0 ? 1.0 / sc : 0.0;
        const T* xc = X + static_cast<int64_t>(c) * p;
        const T* jc = J + static_cast<int64_t>(c) * q;
        // W column -> the p-long factor, J column -> the q-long factor
        double* Wout = trans ? (w.V + static_cast<int64_t>(k) * cols) : (w.U + static_cast<int64_t>(k) * rows);
        double* Jout = trans ? (w.U + static_cast<int64_t>(k) * rows) : (w.V + static_cast<int64_t>(k) * cols);
        for (int r = threadIdx.x; r < p; r += blockDim.x) Wout[r] = static_cast<double>(xc[r]) * inv;
        for (int r = threadIdx.x; r < q; r += blockDim.x) Jout[r] = static_cast<double>(jc[r]);
        if (threadIdx.x == 0) w.sig[k] = sc;
    }
}

// Persistent form: every workgroup takes the next task from the queue until it is empty.
// Tasks are listed largest cost first, so the long blocks start early and the short ones
// fill in behind them. A block whose X and J fit the LDS budget works there, otherwise in
// its global scratch.
template <typename T>
__global__ __launch_bounds__(256) void k_block_svd(const BlockTask* __restrict__ tasks, int ntasks,
                                                   int* __restrict__ counter, int64_t lds_elems,
                                                   int max_sweeps, T tol_scale) {
    extern __shared__ unsigned char smem_raw[];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();   // the previous task is finished with LDS and s_item
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= ntasks) break;
        const BlockTask w = tasks[item];
        const int p = w.rows > w.cols ? w.rows : w.cols;
        const int q = w.rows > w.cols ? w.cols : w.rows;
        const int64_t need = static_cast<int64_t>(p) * q + static_cast<int64_t>(q) * q;
        const T tol = tol_scale * static_cast<T>(p);
        // blocks with more than 256 columns always work in global scratch (their norms and
        // ranks live there too)
        T* X = (need <= lds_elems && q <= 256) ? reinterpret_cast<T*>(smem_raw) : static_cast<T*>(w.scratch);
        T* J = X + static_cast<int64_t>(p) * q;
        block_svd_one<T>(w, X, J, max_sweeps, tol);
    }
}

__global__ __launch_bounds__(256) void k_block_gram_out(const double* __restrict__ lam, const double* __restrict__ E,
                                                        const double* __restrict__ W, int64_t q, int64_t p, int64_t t,
                                                        double cut, double* __restrict__ qout,
                                                        double* __restrict__ pout, double* __restrict__ sig,
                                                        int* __restrict__ status) {
    const int64_t k = blockIdx.y;
    const double l0 = lam[0] > 0 ? lam[0] : 0.0;
    const double lk = lam[k];
    const double lim = cut * cut * l0;
    const double sk = (lk > lim && lk > 0) ? sqrt(lk) : 0.0;
    // a kept singular value under the Gram floor of a non-zero block: warning bit
    if (sk == 0.0 && l0 > 0 && status && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(status, kStatusFloor);
    const double inv = sk > 0 ? 1.0 / sk : 0.0;
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < p + q;
         r += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (r < q)
            qout[k * q + r] = E[r * t + k];
        else
            pout[k * p + (r - q)] = W[(r - q) * t + k] * inv;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) sig[k] = sk;
}

__global__ void k_copy(const double* __restrict__ src, int64_t n, double* __restrict__ dst) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

void launch_copy(const double* src, int64_t n, double* dst, hipStream_t st) {
    if (n <= 0) return;
    const int blocks = static_cast<int>(std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, st, src, n, dst);
}

void launch_block_svd_tasks(bool fp32, const BlockTask* tasks, int ntasks, int* counter, int lds_bytes,
                            int grid, int max_sweeps, double tol_scale, hipStream_t st, KernelTimer* timer) {
    if (ntasks <= 0) return;
    launch_fill_i32(counter, 1, 0, st);
    grid = std::max(1, std::min(grid, ntasks));
    if (fp32) {
        // FP32 rounding bounds what the cosines can reach: a finer scale is taken as FLT_EPSILON
        const int64_t lds_elems = lds_bytes / static_cast<int>(sizeof(float));
        FASTPI_LAUNCH(timer, KT_BLOCK_SVD, k_block_svd<float>, dim3(grid), dim3(256), lds_bytes, st, tasks, ntasks,
                      counter, lds_elems, max_sweeps, static_cast<float>(std::max(tol_scale, static_cast<double>(FLT_EPSILON))));
    } else {
        const int64_t lds_elems = lds_bytes / static_cast<int>(sizeof(double));
        FASTPI_LAUNCH(timer, KT_BLOCK_SVD, k_block_svd<double>, dim3(grid), dim3(256), lds_bytes, st, tasks, ntasks,
                      counter, lds_elems, max_sweeps, tol_scale > 0 ? tol_scale : DBL_EPSILON);
    }
}

void launch_block_gram_out(const double* lam, const double* E, const double* W, int64_t q, int64_t p,
                           int64_t t, double cut, double* qout, double* pout, double* sig, int* status,
                           hipStream_t st) {
    if (t <= 0) return;
    const unsigned gx = static_cast<unsigned>(std::min<int64_t>((p + q + 255) / 256, 64));
    hipLaunchKernelGGL(k_block_gram_out, dim3(gx, static_cast<unsigned>(t)), dim3(256), 0, st, lam, E, W, q, p, t,
                       cut, qout, pout, sig, status);
}

}  // namespace fastpi
