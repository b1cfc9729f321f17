// Dense symmetric eigensolver for the cores of the incremental updates (Eqs. 2 and 3):
// block one-sided Jacobi on the Gram matrix G, FP64.
//
// X starts as G (padded to a multiple of 16 with zero columns). The columns are cut into
// blocks of BW = 16; every round of the round robin pairs the blocks, and for each pair
// (I, J) the 32 x 32 Gram H = [X_I X_J]^T [X_I X_J] is diagonalised by a two-sided Jacobi
// sweep, H = W diag W^T, after which X[:, I u J] <- X[:, I u J] W. X stays equal to G V for
// the orthogonal V that the rotations build; when the columns of X are orthogonal, V
// diagonalises G^2 and hence the positive semidefinite G, so X = V Lambda: the eigenvalues
// are the column norms of X and the eigenvectors its normalised columns (V is never formed).
// A pair whose columns are already orthogonal to `tol` (cosine) is left alone; the sweep
// loop ends after a sweep with no rotated pair.
#include <cfloat>

#include "device_common.h"
#include "kernels.h"

namespace fastpi {

constexpr int BW = 16;
constexpr int PW = 2 * BW;         // columns in a pair
constexpr int GRAM_ROWS = 128;     // rows per partial-Gram workgroup
constexpr int UPD_ROWS = 256;      // rows per update workgroup

__global__ void k_eig_init(const double* __restrict__ G, int64_t q, int64_t ld,
                           double* __restrict__ X) {
    const int64_t n = ld * ld;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int64_t r = e % ld, c = e / ld;
        X[e] = (r < q && c < q) ? G[r * q + c] : 0.0;
    }
}

// floor[0] = (ld eps)^2 ld max_c ||G_c||^2: columns of X = G V whose squared norm is below
// it are rounding noise of a (numerically) zero eigenvalue -- ||x_c|| = lambda_c, whose
// rounding level is ~ ld eps lambda_1, and lambda_1 <= sqrt(ld) max_c ||G_c|| -- and are
// treated as converged (their cosines with anything are meaningless).
__global__ __launch_bounds__(256) void k_eig_floor(const double* __restrict__ norms, int64_t ld,
                                                   double* __restrict__ floor_out) {
    __shared__ double red[256];
    double mx = 0;
    for (int64_t c = threadIdx.x; c < ld; c += blockDim.x) mx = norms[c] > mx ? norms[c] : mx;
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w && red[threadIdx.x + w] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double e = static_cast<double>(ld) * DBL_EPSILON;
        floor_out[0] = isfinite(red[0]) ? e * e * static_cast<double>(ld) * red[0] * red[0] : 0.0;
    }
}

// pair k of step `step` of the round robin over the PW columns of a pair, p < q
__device__ __forceinline__ void inner_pair(int step, int k, int& p, int& q) {
    int a, b;
    if (k == 0) {
        a = PW - 1;
        b = step;
    } else {
        a = step + k;
        if (a >= PW - 1) a -= PW - 1;
        b = step - k;
        if (b < 0) b += PW - 1;
    }
    p = a < b ? a : b;
    q = a < b ? b : a;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Partial Gram of one pair over one row chunk of X.
__global__ __launch_bounds__(256) void k_eig_gram(const double* __restrict__ X, int64_t ld,
                                                  const int2* __restrict__ pairs, int nblk,
                                                  double* __restrict__ Hpart, int nchunk) {
    __shared__ double Y[GRAM_ROWS][PW + 1];
    const int pair = blockIdx.x, ch = blockIdx.y;
    const int2 pb = pairs[pair];
    if (pb.x >= nblk) return;
    const bool hasJ = pb.y < nblk;   // the odd block out is paired with 16 zero columns
    const int64_t r0 = static_cast<int64_t>(ch) * GRAM_ROWS;
    const int nr = static_cast<int>(min<int64_t>(GRAM_ROWS, ld - r0));
    for (int e = threadIdx.x; e < GRAM_ROWS * PW; e += blockDim.x) {
        const int c = e / GRAM_ROWS, r = e % GRAM_ROWS;
        const int col = c < BW ? pb.x * BW + c : pb.y * BW + (c - BW);
        Y[r][c] = (r < nr && (c < BW || hasJ)) ? X[static_cast<int64_t>(col) * ld + r0 + r] : 0.0;
    }
    __syncthreads();
    const int a = threadIdx.x / 8, b0 = (threadIdx.x % 8) * 4;
    double acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
    for (int r = 0; r < nr; ++r) {
        const double ya = Y[r][a];
        acc0 += ya * Y[r][b0];
        acc1 += ya * Y[r][b0 + 1];
        acc2 += ya * Y[r][b0 + 2];
        acc3 += ya * Y[r][b0 + 3];
    }
    double* Hp = Hpart + (static_cast<int64_t>(pair) * nchunk + ch) * (PW * PW) + a * PW + b0;
    Hp[0] = acc0;
    Hp[1] = acc1;
    Hp[2] = acc2;
    Hp[3] = acc3;
}

// Rotation of the symmetric 2x2 [[hpp, hpq], [hpq, hqq]] for the inner sweeps, in FP64 but
// with the hardware reciprocal and reciprocal square root, each refined by Newton steps to
// FP64 accuracy (the IEEE division and square root sequences would sit on the critical path
// of every step). The angle must be FP64-accurate: an angle taken in FP32 leaves couplings of
// about 1e-7 (h_pp - h_qq), which stall the outer iteration on graded Grams.
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = r * (2.0 - x * r);
    return r * (2.0 - x * r);
}
__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * (1.5 - 0.5 * x * y * y);
    return y * (1.5 - 0.5 * x * y * y);
}
__device__ __forceinline__ void fast_rotation(double hpp, double hqq, double hpq, double& c, double& s) {
    c = 1.0;
    s = 0.0;
    const double ahpq = fabs(hpq);
    if (hpq == 0.0 || !(ahpq * ahpq > 0.25 * DBL_EPSILON * DBL_EPSILON * fabs(hpp) * fabs(hqq))) return;
    const double zeta = (hqq - hpp) * rcp_nr(2.0 * hpq);
    const double az = fabs(zeta);
    double t;
    if (az > 1e150) {
        t = 0.5 * rcp_nr(az);
    } else {
        const double x = 1.0 + zeta * zeta;
        t = rcp_nr(az + x * rsq_nr(x));   // 1 / (|zeta| + sqrt(1 + zeta^2))
    }
    if (zeta < 0) t = -t;
    c = rsq_nr(1.0 + t * t);
    s = c * t;
}

// position of index i in the round robin of step `step`: returns its partner and whether
// it is the lower index of its pair
__device__ __forceinline__ void inner_partner(int step, int i, int& partner, bool& lower) {
    int k;
    if (i == PW - 1 || i == step) {
        k = 0;
    } else {
        int d = i - step;
        if (d < 0) d += PW - 1;
        k = d < (PW - 1) - d ? d : (PW - 1) - d;
    }
    int p, q;
    inner_pair(step, k, p, q);
    lower = (i == p);
    partner = lower ? q : p;
}

// Slot permutation between inner steps. Slots 0..31 hold the 32 columns of a pair; step
// pairs are always the adjacent slots (2k, 2k+1). Slot 0 keeps the fixed player of the
// circle-method round robin, slot 1 the player at circle offset 0 and slots 2d, 2d+1 the
// players at offsets +d and -d; a step moves every circle player one offset down, so the
// next step pairs the next round-robin partners. After 31 steps every slot is back home.
__device__ __forceinline__ int inner_next_slot(int x) {
    if (x == 0) return 0;
    if (x == 1) return 3;
    if (x == 2) return 1;
    if ((x & 1) == 0) return x - 2;   // offset +d -> +(d-1)
    if (x == PW - 1) return PW - 2;   // offset -15 -> +15
    return x + 2;                     // offset -d -> -(d+1)
}

// One workgroup of 256 threads per pair. Thread (a, b) keeps the 2x2 blocks
// H[2a:2a+2][2b:2b+2] and W[2a:2a+2][2b:2b+2] in registers (H indexed by slots on both
// sides, W by input column and slot). In a step the 16 diagonal threads compute the rotation
// of their slot pair, every thread applies J_a^T (.) J_b to its H block and (.) J_b to its W
// block in registers, and the blocks are scattered to their next slots through LDS.
__global__ __launch_bounds__(256) void k_eig_solve(const double* __restrict__ Hpart, int nchunk,
                                                   const int2* __restrict__ pairs, int nblk,
                                                   double* __restrict__ Wout,
                                                   int* __restrict__ flag,
                                                   int* __restrict__ rot_count, double tol,
                                                   int inner_sweeps,
                                                   const double* __restrict__ noise_floor) {
    __shared__ double Hs[2][PW][PW + 1];
    __shared__ double Ws[2][PW][PW + 1];
    __shared__ double rot[PW / 2][2];
    __shared__ int s_need;
    const int pair = blockIdx.x;
    const int2 pb = pairs[pair];
    if (pb.x >= nblk) {
        if (threadIdx.x == 0) flag[pair] = 0;
        return;
    }
    const double* Hp = Hpart + static_cast<int64_t>(pair) * nchunk * (PW * PW);
    for (int e = threadIdx.x; e < PW * PW; e += 256) {
        double acc = 0;
        for (int c = 0; c < nchunk; ++c) acc += Hp[static_cast<int64_t>(c) * PW * PW + e];
        Hs[0][e / PW][e % PW] = acc;
    }
    if (threadIdx.x == 0) s_need = 0;
    __syncthreads();
    const double nf = noise_floor[0];
    {
        int need = 0;
        for (int e = threadIdx.x; e < PW * PW; e += 256) {
            const int i = e / PW, j = e % PW;
            if (i < j) {
                const double hii = Hs[0][i][i], hjj = Hs[0][j][j], hij = Hs[0][i][j];
                if (hii > nf && hjj > nf && fabs(hij) > tol * sqrt(hii) * sqrt(hjj)) need = 1;
            }
        }
        if (need) s_need = 1;
    }
    __syncthreads();
    if (!s_need) {
        if (threadIdx.x == 0) flag[pair] = 0;
        return;
    }
    const int a = threadIdx.x / (PW / 2), b = threadIdx.x % (PW / 2);
    const int r0 = 2 * a, r1 = 2 * a + 1, c0 = 2 * b, c1 = 2 * b + 1;
    double h00 = Hs[0][r0][c0], h01 = Hs[0][r0][c1], h10 = Hs[0][r1][c0], h11 = Hs[0][r1][c1];
    double w00 = (r0 == c0), w01 = (r0 == c1), w10 = (r1 == c0), w11 = (r1 == c1);
    // slot permutation of the four rows/columns this thread owns
    const int pr0 = inner_next_slot(r0), pr1 = inner_next_slot(r1);
    const int pc0 = inner_next_slot(c0), pc1 = inner_next_slot(c1);
    int buf = 1;
    for (int sw = 0; sw < inner_sweeps; ++sw) {
        for (int step = 0; step < PW - 1; ++step) {
            if (a == b) {
                double c = 1.0, s = 0.0;
                if (h00 > nf && h11 > nf) fast_rotation(h00, h11, h01, c, s);
                rot[a][0] = c;
                rot[a][1] = s;
            }
            __syncthreads();
            const double ca = rot[a][0], sa = rot[a][1], cb = rot[b][0], sb = rot[b][1];
            // rows: new row p = c row_p - s row_q, new row q = s row_p + c row_q
            const double x00 = ca * h00 - sa * h10, x01 = ca * h01 - sa * h11;
            const double x10 = sa * h00 + ca * h10, x11 = sa * h01 + ca * h11;
            // columns, likewise
            h00 = cb * x00 - sb * x01;
            h01 = sb * x00 + cb * x01;
            h10 = cb * x10 - sb * x11;
            h11 = sb * x10 + cb * x11;
            const double y00 = cb * w00 - sb * w01, y01 = sb * w00 + cb * w01;
            const double y10 = cb * w10 - sb * w11, y11 = sb * w10 + cb * w11;
            w00 = y00;
            w01 = y01;
            w10 = y10;
            w11 = y11;
            // move to the next step's slots (W rows are input columns and stay)
            Hs[buf][pr0][pc0] = h00;
            Hs[buf][pr0][pc1] = h01;
            Hs[buf][pr1][pc0] = h10;
            Hs[buf][pr1][pc1] = h11;
            Ws[buf][r0][pc0] = w00;
            Ws[buf][r0][pc1] = w01;
            Ws[buf][r1][pc0] = w10;
            Ws[buf][r1][pc1] = w11;
            __syncthreads();
            h00 = Hs[buf][r0][c0];
            h01 = Hs[buf][r0][c1];
            h10 = Hs[buf][r1][c0];
            h11 = Hs[buf][r1][c1];
            w00 = Ws[buf][r0][c0];
            w01 = Ws[buf][r0][c1];
            w10 = Ws[buf][r1][c0];
            w11 = Ws[buf][r1][c1];
            buf ^= 1;
        }
    }
    // after whole sweeps every slot holds its own column again
    double* Wg = Wout + static_cast<int64_t>(pair) * PW * PW;
    Wg[r0 * PW + c0] = w00;
    Wg[r0 * PW + c1] = w01;
    Wg[r1 * PW + c0] = w10;
    Wg[r1 * PW + c1] = w11;
    if (threadIdx.x == 0) {
        flag[pair] = 1;
        atomicAdd(rot_count, 1);
    }
}

// X[:, I u J] <- X[:, I u J] W, one thread per row
__global__ __launch_bounds__(UPD_ROWS) void k_eig_update(double* __restrict__ X, int64_t ld,
                                                         const int2* __restrict__ pairs, int nblk,
                                                         const double* __restrict__ Wall,
                                                         const int* __restrict__ flag) {
    __shared__ double W[PW][PW];
    const int pair = blockIdx.x;
    const int2 pb = pairs[pair];
    if (pb.x >= nblk) return;
    if (flag[pair] == 0) return;
    const bool hasJ = pb.y < nblk;
    const double* Wg = Wall + static_cast<int64_t>(pair) * PW * PW;
    for (int e = threadIdx.x; e < PW * PW; e += blockDim.x) W[e / PW][e % PW] = Wg[e];
    __syncthreads();
    const int64_t r = static_cast<int64_t>(blockIdx.y) * UPD_ROWS + threadIdx.x;
    if (r >= ld) return;
    double y[PW];
#pragma unroll
    for (int c = 0; c < PW; ++c) {
        const int col = c < BW ? pb.x * BW + c : pb.y * BW + (c - BW);
        y[c] = (c < BW || hasJ) ? X[static_cast<int64_t>(col) * ld + r] : 0.0;
    }
    const int jend = hasJ ? PW : BW;
#pragma unroll 4
    for (int j = 0; j < jend; ++j) {
        double acc = 0;
#pragma unroll
        for (int k = 0; k < PW; ++k) acc += y[k] * W[k][j];
        const int col = j < BW ? pb.x * BW + j : pb.y * BW + (j - BW);
        X[static_cast<int64_t>(col) * ld + r] = acc;
    }
}

// eigenvalues: column norms of X (non-finite values sort last so the order stays a
// permutation)
__global__ void k_eig_norms(const double* __restrict__ X, int64_t ld, int64_t q,
                            double* __restrict__ lam) {
    const int lane = threadIdx.x % kWave;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (c >= ld) return;
    double acc = 0;
    for (int64_t r = lane; r < q; r += kWave) {
        const double v = X[c * ld + r];
        acc += v * v;
    }
    acc = wave_sum(acc);
    if (lane == 0) lam[c] = (c < q && isfinite(acc)) ? sqrt(acc) : -DBL_MAX;
}

// order of the t largest eigenvalues (descending, ties to the lower column)
__global__ __launch_bounds__(1024) void k_eig_select(const double* __restrict__ lam, int64_t q,
                                                     int64_t t, int* __restrict__ order) {
    for (int64_t c = threadIdx.x; c < q; c += blockDim.x) {
        const double lc = lam[c];
        int64_t rk = 0;
        for (int64_t d = 0; d < q; ++d) {
            const double ld_ = lam[d];
            rk += (ld_ > lc) || (ld_ == lc && d < c);
        }
        if (rk < t) order[rk] = static_cast<int>(c);
    }
}

// vecs (q x t, row-major): the normalised columns of X; vals (t): their norms
__global__ void k_eig_output(const double* __restrict__ X, int64_t ld, int64_t q, int64_t t,
                             const int* __restrict__ order, const double* __restrict__ lam,
                             double* __restrict__ vals, double* __restrict__ vecs) {
    const int64_t n = q * t;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int64_t r = e / t, k = e % t;
        const double l = lam[order[k]];
        const double inv = l > 0 ? 1.0 / l : 0.0;
        vecs[e] = X[static_cast<int64_t>(order[k]) * ld + r] * inv;
        if (r == 0) vals[k] = l > 0 ? l : 0.0;
    }
}

int64_t eig_padded_order(int64_t q) { return ((q + BW - 1) / BW) * BW; }

size_t eig_workspace_doubles(int64_t q) {
    const int64_t ld = eig_padded_order(q);
    const int64_t nblk = ld / BW;
    const int64_t npairs = (nblk + 1) / 2;
    const int64_t nchunk = (ld + GRAM_ROWS - 1) / GRAM_ROWS;
    return static_cast<size_t>(ld * ld + npairs * nchunk * PW * PW + npairs * PW * PW + 2 * ld + 64);
}

size_t eig_int_workspace(int64_t q, int max_sweeps) {
    const int64_t ld = eig_padded_order(q);
    const int64_t npairs = (ld / BW + 1) / 2;
    return static_cast<size_t>(2 * npairs + ld + max_sweeps + 64);
}

// Host driver. ws holds eig_workspace_doubles(q) doubles, iws eig_int_workspace(q, max_sweeps)
// ints; pair_tables is the device copy of the round-robin tables for the padded order.
// The rotation count of sweep k is read back while sweep k+1 is already queued, so the
// device never waits on the host; a sweep queued after convergence finds nothing to do.
int eig_top(const double* G, int64_t q, int64_t t, double* vals, double* vecs, double* ws,
            int* iws, const int2* pair_tables, int max_sweeps, double tol, int inner_sweeps,
            int* sweeps_out, int* host_counter, hipStream_t st, hipStream_t copy_st,
            KernelTimer* timer) {
    const int64_t ld = eig_padded_order(q);
    const int nblk = static_cast<int>(ld / BW);
    const int nbe = nblk + (nblk & 1);     // even number of slots (the extra one is a dummy)
    const int npairs = nbe / 2;
    const int rounds = nbe - 1;
    const int nchunk = static_cast<int>((ld + GRAM_ROWS - 1) / GRAM_ROWS);
    const int nupd = static_cast<int>((ld + UPD_ROWS - 1) / UPD_ROWS);
    double* X = ws;
    double* Hpart = X + ld * ld;
    double* W = Hpart + static_cast<int64_t>(npairs) * nchunk * PW * PW;
    double* lam = W + static_cast<int64_t>(npairs) * PW * PW;
    int* flag = iws;
    int* arrive = flag + npairs;
    int* order = arrive + npairs;
    int* rot = order + ld;                 // one counter per sweep
    // reads the rotation counter of sweep k on the side stream once sweep k has finished
    auto read_counter = [&](int k, hipEvent_t e) -> int {
        if (hipStreamWaitEvent(copy_st, e, 0) != hipSuccess) return FASTPI_EHIP;
        if (hipMemcpyAsync(host_counter, rot + k, sizeof(int), hipMemcpyDeviceToHost, copy_st) != hipSuccess)
            return FASTPI_EHIP;
        if (hipStreamSynchronize(copy_st) != hipSuccess) return FASTPI_EHIP;
        return FASTPI_OK;
    };
    hipLaunchKernelGGL(k_eig_init, dim3(static_cast<int>(std::min<int64_t>((ld * ld + 255) / 256, 8192))),
                       dim3(256), 0, st, G, q, ld, X);
    launch_fill_i32(rot, max_sweeps, 0, st);
    hipLaunchKernelGGL(k_eig_norms, dim3(static_cast<int>((ld + 3) / 4)), dim3(256), 0, st, X, ld, q, lam);
    hipLaunchKernelGGL(k_eig_floor, dim3(1), dim3(256), 0, st, lam, ld, lam + ld);
    if (tol <= 0) tol = static_cast<double>(ld) * DBL_EPSILON;
    hipEvent_t ev[2];
    if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess) return FASTPI_EHIP;
    if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) return FASTPI_EHIP;
    int sweeps_done = 0;
    bool converged = false;
    int checked = 0;   // sweeps whose counter has been read
    for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
        for (int round = 0; round < rounds; ++round) {
            const int2* pr = pair_tables + static_cast<int64_t>(round) * npairs;
            long ts = timer ? timer->begin(KT_EIG_GRAM, st) : -1;
            hipLaunchKernelGGL(k_eig_gram, dim3(npairs, nchunk), dim3(256), 0, st, X, ld, pr, nblk, Hpart,
                               nchunk);
            if (timer) timer->end(ts, st);
            ts = timer ? timer->begin(KT_EIG_SOLVE, st) : -1;
            hipLaunchKernelGGL(k_eig_solve, dim3(npairs), dim3(256), 0, st, Hpart, nchunk, pr, nblk, W,
                               flag, rot + sweep, tol, inner_sweeps, lam + ld);
            if (timer) timer->end(ts, st);
            ts = timer ? timer->begin(KT_EIG_UPDATE, st) : -1;
            hipLaunchKernelGGL(k_eig_update, dim3(npairs, nupd), dim3(UPD_ROWS), 0, st, X, ld, pr, nblk,
                               W, flag);
            if (timer) timer->end(ts, st);
        }
        hipEventRecord(ev[sweep & 1], st);
        sweeps_done = sweep + 1;
        if (sweep >= 1) {
            // read the previous sweep's counter while this one runs
            if (read_counter(sweep - 1, ev[(sweep - 1) & 1]) != FASTPI_OK) return FASTPI_EHIP;
            checked = sweep;
            if (*host_counter == 0) converged = true;
        }
    }
    if (!converged && checked < sweeps_done) {
        if (read_counter(sweeps_done - 1, ev[(sweeps_done - 1) & 1]) != FASTPI_OK) return FASTPI_EHIP;
        if (*host_counter == 0) converged = true;
    }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (sweeps_out) *sweeps_out = sweeps_done;
    hipLaunchKernelGGL(k_eig_norms, dim3(static_cast<int>((ld + 3) / 4)), dim3(256), 0, st, X, ld, q, lam);
    hipLaunchKernelGGL(k_eig_select, dim3(1), dim3(1024), 0, st, lam, q, t, order);
    hipLaunchKernelGGL(k_eig_output, dim3(static_cast<int>(std::min<int64_t>((q * t + 255) / 256, 8192))),
                       dim3(256), 0, st, X, ld, q, t, order, lam, vals, vecs);
    return converged ? FASTPI_OK : FASTPI_ENOCONV;
}

// circle-method tables for nblk blocks: rounds x npairs entries (dummy slot = nblk)
void eig_pair_table(int64_t q, std::vector<int2>& out) {
    const int64_t ld = eig_padded_order(q);
    const int nblk = static_cast<int>(ld / BW);
    const int nbe = nblk + (nblk & 1);
    const int npairs = nbe / 2;
    out.clear();
    for (int round = 0; round < nbe - 1; ++round) {
        for (int pr = 0; pr < npairs; ++pr) {
            int a, b;
            if (pr == 0) {
                a = nbe - 1;
                b = round;
            } else {
                a = (round + pr) % (nbe - 1);
                b = (round - pr + nbe - 1) % (nbe - 1);
            }
            if (a > b) std::swap(a, b);
            out.push_back(make_int2(a, b));
        }
    }
}

}  // namespace fastpi
