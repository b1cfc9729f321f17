// Dense symmetric eigensolver for the cores of the incremental updates (Eqs. 2 and 3):
// block one-sided Jacobi on the Gram matrix G, FP64.
//
// X starts as G (padded to a multiple of 16 with zero columns) and V as I. The columns are
// cut into blocks of BW = 16; every round of the round robin pairs the blocks, and for each
// pair (I, J) the 32 x 32 Gram H = [X_I X_J]^T [X_I X_J] is diagonalised by a two-sided
// Jacobi sweep, H = W diag W^T, after which X[:, I u J] <- X[:, I u J] W and
// V[:, I u J] <- V[:, I u J] W. At convergence the columns of X = G V are orthogonal, so V
// holds eigenvectors of G, and the eigenvalues are the Rayleigh quotients v_c^T x_c.
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
                           double* __restrict__ X, double* __restrict__ V) {
    const int64_t n = ld * ld;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int64_t r = e % ld, c = e / ld;
        X[e] = (r < q && c < q) ? G[r * q + c] : 0.0;
        V[e] = (r == c) ? 1.0 : 0.0;
    }
}

// partial Gram of one pair over one row chunk
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
    double* H = Hpart + (static_cast<int64_t>(pair) * nchunk + ch) * (PW * PW) + a * PW + b0;
    H[0] = acc0;
    H[1] = acc1;
    H[2] = acc2;
    H[3] = acc3;
}

// sum the partials of one pair, test orthogonality, diagonalise with one or more Jacobi
// sweeps (16 disjoint rotations per step), write W
__global__ __launch_bounds__(64) void k_eig_solve(const double* __restrict__ Hpart, int nchunk,
                                                  const int2* __restrict__ pairs, int nblk,
                                                  double* __restrict__ Wout, int* __restrict__ flag,
                                                  int* __restrict__ rot_count, double tol,
                                                  int inner_sweeps) {
    __shared__ double H[PW][PW + 1];
    __shared__ double W[PW][PW + 1];
    __shared__ double cs[PW / 2][3];
    __shared__ int s_need;
    const int pair = blockIdx.x;
    const int2 pb = pairs[pair];
    const int lane = threadIdx.x;
    if (pb.x >= nblk) {
        if (lane == 0) flag[pair] = 0;
        return;
    }
    const double* Hp = Hpart + static_cast<int64_t>(pair) * nchunk * (PW * PW);
    for (int e = lane; e < PW * PW; e += 64) {
        double acc = 0;
        for (int c = 0; c < nchunk; ++c) acc += Hp[static_cast<int64_t>(c) * PW * PW + e];
        H[e / PW][e % PW] = acc;
        W[e / PW][e % PW] = (e / PW == e % PW) ? 1.0 : 0.0;
    }
    if (lane == 0) s_need = 0;
    __syncthreads();
    // off-diagonal test in the cosine sense
    int need = 0;
    for (int e = lane; e < PW * PW; e += 64) {
        const int i = e / PW, j = e % PW;
        if (i < j) {
            const double hii = H[i][i], hjj = H[j][j], hij = H[i][j];
            if (hii > 0 && hjj > 0 && fabs(hij) > tol * sqrt(hii) * sqrt(hjj)) need = 1;
        }
    }
    if (need) s_need = 1;
    __syncthreads();
    if (!s_need) {
        if (lane == 0) flag[pair] = 0;
        return;
    }
    for (int sw = 0; sw < inner_sweeps; ++sw) {
        for (int step = 0; step < PW - 1; ++step) {
            if (lane < PW / 2) {
                int p, q;
                round_robin_pair(step, lane, PW, p, q);
                const double hpp = H[p][p], hqq = H[q][q], hpq = H[p][q];
                double c = 1, s = 0, t = 0;
                if (hpq != 0.0 && fabs(hpq) > 0.5 * DBL_EPSILON * sqrt(fabs(hpp)) * sqrt(fabs(hqq)))
                    jacobi_rotation(hpp, hqq, hpq, c, s, t);
                cs[lane][0] = c;
                cs[lane][1] = s;
                cs[lane][2] = t;
            }
            __syncthreads();
            // rows: H <- J^T H
            for (int e = lane; e < (PW / 2) * PW; e += 64) {
                const int k = e / PW, j = e % PW;
                int p, q;
                round_robin_pair(step, k, PW, p, q);
                const double c = cs[k][0], s = cs[k][1];
                const double hp = H[p][j], hq = H[q][j];
                H[p][j] = c * hp - s * hq;
                H[q][j] = s * hp + c * hq;
            }
            __syncthreads();
            // columns: H <- H J, W <- W J
            for (int e = lane; e < (PW / 2) * PW; e += 64) {
                const int k = e / PW, i = e % PW;
                int p, q;
                round_robin_pair(step, k, PW, p, q);
                const double c = cs[k][0], s = cs[k][1];
                const double hp = H[i][p], hq = H[i][q];
                H[i][p] = c * hp - s * hq;
                H[i][q] = s * hp + c * hq;
                const double wp = W[i][p], wq = W[i][q];
                W[i][p] = c * wp - s * wq;
                W[i][q] = s * wp + c * wq;
            }
            __syncthreads();
            if (lane < PW / 2 && cs[lane][1] != 0.0) {
                int p, q;
                round_robin_pair(step, lane, PW, p, q);
                H[p][q] = 0.0;
                H[q][p] = 0.0;
            }
            __syncthreads();
        }
    }
    double* Wg = Wout + static_cast<int64_t>(pair) * PW * PW;
    for (int e = lane; e < PW * PW; e += 64) Wg[e] = W[e / PW][e % PW];
    if (lane == 0) {
        flag[pair] = 1;
        atomicAdd(rot_count, 1);
    }
}

// X[:, I u J] <- X[:, I u J] W and V likewise (blockIdx.z selects X or V)
__global__ __launch_bounds__(UPD_ROWS) void k_eig_update(double* __restrict__ X, double* __restrict__ V,
                                                         int64_t ld, const int2* __restrict__ pairs,
                                                         int nblk, const double* __restrict__ Wall,
                                                         const int* __restrict__ flag) {
    __shared__ double W[PW][PW];
    const int pair = blockIdx.x;
    const int2 pb = pairs[pair];
    if (pb.x >= nblk) return;
    if (flag[pair] == 0) return;
    const bool hasJ = pb.y < nblk;
    double* M = blockIdx.z == 0 ? X : V;
    const double* Wg = Wall + static_cast<int64_t>(pair) * PW * PW;
    for (int e = threadIdx.x; e < PW * PW; e += blockDim.x) W[e / PW][e % PW] = Wg[e];
    __syncthreads();
    const int64_t r = static_cast<int64_t>(blockIdx.y) * UPD_ROWS + threadIdx.x;
    if (r >= ld) return;
    double y[PW];
#pragma unroll
    for (int c = 0; c < PW; ++c) {
        const int col = c < BW ? pb.x * BW + c : pb.y * BW + (c - BW);
        y[c] = (c < BW || hasJ) ? M[static_cast<int64_t>(col) * ld + r] : 0.0;
    }
    const int jend = hasJ ? PW : BW;
#pragma unroll 4
    for (int j = 0; j < jend; ++j) {
        double acc = 0;
#pragma unroll
        for (int k = 0; k < PW; ++k) acc += y[k] * W[k][j];
        const int col = j < BW ? pb.x * BW + j : pb.y * BW + (j - BW);
        M[static_cast<int64_t>(col) * ld + r] = acc;
    }
}

// eigenvalue estimates: Rayleigh quotients v_c^T x_c (x_c = G v_c)
__global__ void k_eig_rayleigh(const double* __restrict__ X, const double* __restrict__ V,
                               int64_t ld, int64_t q, double* __restrict__ lam) {
    const int lane = threadIdx.x % kWave;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (c >= ld) return;
    double acc = 0;
    for (int64_t r = lane; r < q; r += kWave) acc += V[c * ld + r] * X[c * ld + r];
    acc = wave_sum(acc);
    // non-finite values (from a non-finite input) sort last, keeping the order a permutation
    if (lane == 0) lam[c] = (c < q && isfinite(acc)) ? acc : -DBL_MAX;
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

// vecs (q x t, row-major) and vals (t)
__global__ void k_eig_output(const double* __restrict__ V, int64_t ld, int64_t q, int64_t t,
                             const int* __restrict__ order, const double* __restrict__ lam,
                             double* __restrict__ vals, double* __restrict__ vecs) {
    const int64_t n = q * t;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int64_t r = e / t, k = e % t;
        vecs[e] = V[static_cast<int64_t>(order[k]) * ld + r];
        if (r == 0) vals[k] = lam[order[k]];
    }
}

int64_t eig_padded_order(int64_t q) { return ((q + BW - 1) / BW) * BW; }

size_t eig_workspace_doubles(int64_t q) {
    const int64_t ld = eig_padded_order(q);
    const int64_t nblk = ld / BW;
    const int64_t npairs = (nblk + 1) / 2;
    const int64_t nchunk = (ld + GRAM_ROWS - 1) / GRAM_ROWS;
    return static_cast<size_t>(2 * ld * ld + npairs * nchunk * PW * PW + npairs * PW * PW + 2 * ld + 64);
}

// Host driver. ws holds eig_workspace_doubles(q) doubles; iws holds ints for flags and the
// ordering; pair_tables is the device copy of the round-robin tables for nblk blocks.
int eig_top(const double* G, int64_t q, int64_t t, double* vals, double* vecs, double* ws,
            int* iws, const int2* pair_tables, int max_sweeps, double tol, int inner_sweeps,
            int* sweeps_out, int* host_counter, hipStream_t st) {
    const int64_t ld = eig_padded_order(q);
    const int nblk = static_cast<int>(ld / BW);
    const int nbe = nblk + (nblk & 1);     // even number of slots (the extra one is a dummy)
    const int npairs = nbe / 2;
    const int rounds = nbe - 1;
    const int nchunk = static_cast<int>((ld + GRAM_ROWS - 1) / GRAM_ROWS);
    const int nupd = static_cast<int>((ld + UPD_ROWS - 1) / UPD_ROWS);
    double* X = ws;
    double* V = X + ld * ld;
    double* Hpart = V + ld * ld;
    double* W = Hpart + static_cast<int64_t>(npairs) * nchunk * PW * PW;
    double* lam = W + static_cast<int64_t>(npairs) * PW * PW;
    int* flag = iws;
    int* rot = flag + npairs;
    int* order = rot + 4;
    hipLaunchKernelGGL(k_eig_init, dim3(static_cast<int>(std::min<int64_t>((ld * ld + 255) / 256, 8192))),
                       dim3(256), 0, st, G, q, ld, X, V);
    if (tol <= 0) tol = static_cast<double>(ld) * DBL_EPSILON;
    int sweep = 0;
    bool converged = nblk <= 0;
    for (; sweep < max_sweeps && !converged; ++sweep) {
        launch_fill_i32(rot, 1, 0, st);
        for (int round = 0; round < rounds; ++round) {
            const int2* pr = pair_tables + static_cast<int64_t>(round) * npairs;
            hipLaunchKernelGGL(k_eig_gram, dim3(npairs, nchunk), dim3(256), 0, st, X, ld, pr, nblk,
                               Hpart, nchunk);
            hipLaunchKernelGGL(k_eig_solve, dim3(npairs), dim3(64), 0, st, Hpart, nchunk, pr, nblk,
                               W, flag, rot, tol, inner_sweeps);
            hipLaunchKernelGGL(k_eig_update, dim3(npairs, nupd, 2), dim3(UPD_ROWS), 0, st, X, V, ld,
                               pr, nblk, W, flag);
        }
        if (hipMemcpyAsync(host_counter, rot, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
            return FASTPI_EHIP;
        if (hipStreamSynchronize(st) != hipSuccess) return FASTPI_EHIP;
        if (*host_counter == 0) converged = true;
    }
    if (sweeps_out) *sweeps_out = sweep;
    hipLaunchKernelGGL(k_eig_rayleigh, dim3(static_cast<int>((ld + 3) / 4)), dim3(256), 0, st, X, V, ld,
                       q, lam);
    hipLaunchKernelGGL(k_eig_select, dim3(1), dim3(1024), 0, st, lam, q, t, order);
    hipLaunchKernelGGL(k_eig_output, dim3(static_cast<int>(std::min<int64_t>((q * t + 255) / 256, 8192))),
                       dim3(256), 0, st, V, ld, q, t, order, lam, vals, vecs);
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
