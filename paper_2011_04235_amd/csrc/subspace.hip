// Dense kernels of the subspace core solver (the top-t eigenpairs of an update's Gram
// matrix G by subspace iteration, Rayleigh-Ritz on the converged basis): the Cholesky QR
// that orthonormalises the iterate (B = Y^T Y = L L^T, Q = Y L^-T) and the residual check of
// the final eigenpairs. Everything is batched over the cores of one update step ("jobs"):
// one launch per kernel and panel for all of them.
//
// Cholesky: right-looking, panels of 32 columns, in place on the lower triangle of B
// (kp x kp row-major, kp = 32 * 2^j >= k). Per panel, one kernel factors the 32 x 32
// diagonal block in LDS (every workgroup of the launch does it, each then solves its own
// chunk of rows below, x L11^T = b, so no second launch is needed for the panel's rows), and
// a 64 x 64-tiled kernel subtracts L21 L21^T from the lower triangle of the trailing matrix.
// A pivot whose square falls to kc * eps of its column's original diagonal marks the job
// (the iterate lost rank numerically); the caller then takes the Jacobi route instead.
//
// Inverse L^-1: the 32 x 32 diagonal blocks are inverted in LDS, then recursive doubling
// over levels s = 32, 64, ..: the off-diagonal block of a 2s x 2s diagonal block is
// -D^-1 (C A^-1) (A^-1, D^-1 from the level below, C the block of L), two small GEMMs per
// pair, batched over pairs and jobs. Rows and columns between k and kp are the identity.
#include <cfloat>

#include "device_common.h"
#include "kernels.h"

namespace fastpi {

constexpr int CP = 32;    // panel width / diagonal block of the inverse
constexpr int CT = 64;    // tile of the trailing update and of the inverse products

// original diagonal of every job's B (the reference of the rank test)
__global__ void k_chol_diag(const CholJob* __restrict__ jobs) {
    const CholJob& J = jobs[blockIdx.y];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < J.kc; i += gridDim.x * blockDim.x)
        J.dg[i] = J.B[static_cast<int64_t>(i) * J.kp + i];
}

// Panel [c0, c0 + 32): factor the diagonal block, then rows [c0 + 32 + 256 * blockIdx.x, ..)
// of the panel by forward substitution against L11.
__global__ __launch_bounds__(256) void k_chol_panel(const CholJob* __restrict__ jobs, int c0) {
    const CholJob& J = jobs[blockIdx.y];
    const int kc = J.kc, kp = J.kp;
    if (c0 >= kc) return;
    const int tid = threadIdx.x;
    const int row = c0 + CP + static_cast<int>(blockIdx.x) * 256 + tid;
    if (blockIdx.x > 0 && c0 + CP + static_cast<int>(blockIdx.x) * 256 >= kc) return;
    __shared__ double D[CP][CP + 1];
    __shared__ int bad;
    double* B = J.B;
    for (int e = tid; e < CP * CP; e += 256) {
        const int i = e / CP, j = e % CP;
        D[i][j] = B[static_cast<int64_t>(c0 + i) * kp + c0 + j];
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    const double lim = static_cast<double>(kc) * DBL_EPSILON;
    for (int c = 0; c < CP; ++c) {
        if (tid == 0) {
            double d = D[c][c];
            if (!(d > lim * J.dg[c0 + c])) {
                bad = 1;
                d = 1.0;   // keeps the arithmetic finite; the job is marked
            }
            D[c][c] = sqrt(d);
        }
        __syncthreads();
        if (tid > c && tid < CP) D[tid][c] /= D[c][c];
        __syncthreads();
        for (int e = tid; e < CP * CP; e += 256) {
            const int i = e / CP, j = e % CP;
            if (j > c && i >= j) D[i][j] -= D[i][c] * D[j][c];
        }
        __syncthreads();
    }
    // L11 goes to the job's stack of diagonal blocks, not into B: the other workgroups of this
    // launch still read B's diagonal block
    if (blockIdx.x == 0) {
        for (int e = tid; e < CP * CP; e += 256) {
            const int i = e / CP, j = e % CP;
            J.Ld[static_cast<int64_t>(c0 + i) * CP + j] = (j <= i) ? D[i][j] : 0.0;
        }
        if (tid == 0 && bad) atomicOr(J.flag, 1);
    }
    if (row >= kc) return;
    double x[CP];
    double* br = B + static_cast<int64_t>(row) * kp + c0;
#pragma unroll
    for (int j = 0; j < CP; ++j) x[j] = br[j];
#pragma unroll
    for (int j = 0; j < CP; ++j) {
        double v = x[j];
#pragma unroll
        for (int l = 0; l < j; ++l) v -= x[l] * D[j][l];
        x[j] = v / D[j][j];
    }
#pragma unroll
    for (int j = 0; j < CP; ++j) br[j] = x[j];
}

// B[i][j] -= sum_l L[i][c0+32+.. ] ... : the trailing lower triangle [c1, kc)^2, c1 = c0 + 32,
// minus L21 L21^T with L21 = B[c1:kc, c0:c0+32]. Tiles (ti, tj), tj <= ti, numbered
// row by row of the lower triangle.
__global__ __launch_bounds__(256) void k_chol_update(const CholJob* __restrict__ jobs, int c0) {
    const CholJob& J = jobs[blockIdx.y];
    const int kc = J.kc, kp = J.kp;
    const int c1 = c0 + CP;
    if (c1 >= kc) return;
    const int nt = (kc - c1 + CT - 1) / CT;
    const int tri = static_cast<int>(blockIdx.x);
    if (tri >= nt * (nt + 1) / 2) return;
    int ti = static_cast<int>((sqrt(8.0 * tri + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= tri) ++ti;
    while (ti * (ti + 1) / 2 > tri) --ti;
    const int tj = tri - ti * (ti + 1) / 2;
    const int i0 = c1 + ti * CT, j0 = c1 + tj * CT;
    __shared__ double Li[CP][CT + 1];
    __shared__ double Lj[CP][CT + 1];
    double* B = J.B;
    for (int e = threadIdx.x; e < CP * CT; e += 256) {
        const int t = e / CP, l = e % CP;
        Li[l][t] = (i0 + t < kc) ? B[static_cast<int64_t>(i0 + t) * kp + c0 + l] : 0.0;
        Lj[l][t] = (j0 + t < kc) ? B[static_cast<int64_t>(j0 + t) * kp + c0 + l] : 0.0;
    }
    __syncthreads();
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4] = {};
#pragma unroll 8
    for (int l = 0; l < CP; ++l) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = Li[l][ty * 4 + u];
            b[u] = Lj[l][tx * 4 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = i0 + ty * 4 + u;
        if (i >= kc) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + tx * 4 + v;
            if (j < kc && j <= i) B[static_cast<int64_t>(i) * kp + j] -= acc[u][v];
        }
    }
}

// Linv's 32 x 32 diagonal blocks: the inverse of L's (lower triangular) diagonal blocks
// (the panels' stack Ld), one wave per block, lane j computing column j by forward
// substitution. Blocks at or past kc hold the identity (Ld is the identity there).
__global__ __launch_bounds__(64) void k_trinv_diag(const CholJob* __restrict__ jobs) {
    const CholJob& J = jobs[blockIdx.y];
    const int kp = J.kp;
    const int b0 = static_cast<int>(blockIdx.x) * CP;
    if (b0 >= kp) return;
    __shared__ double L[CP][CP + 1];
    __shared__ double X[CP][CP + 1];
    const int tid = threadIdx.x;
    for (int e = tid; e < CP * CP; e += 64) {
        const int i = e / CP, j = e % CP;
        L[i][j] = (j <= i) ? J.Ld[static_cast<int64_t>(b0 + i) * CP + j] : 0.0;
    }
    __syncthreads();
    if (tid < CP) {
        const int j = tid;
        for (int i = 0; i < j; ++i) X[i][j] = 0.0;
        X[j][j] = 1.0 / L[j][j];
        for (int i = j + 1; i < CP; ++i) {
            double v = 0.0;
            for (int l = j; l < i; ++l) v += L[i][l] * X[l][j];
            X[i][j] = -v / L[i][i];
        }
    }
    __syncthreads();
    for (int e = tid; e < CP * CP; e += 64) {
        const int i = e / CP, j = e % CP;
        J.Linv[static_cast<int64_t>(b0 + i) * kp + b0 + j] = X[i][j];
    }
}

// One product of a doubling level s for every pair p (rows i1 = (2p+1) s, columns i0 = 2p s):
// phase 0: T_p = L[i1:, i0:] Linv[i0:, i0:]; phase 1: Linv[i1:, i0:] = -Linv[i1:, i1:] T_p.
// Pairs whose second block starts at or past kc keep a zero block.
__global__ __launch_bounds__(256) void k_trinv_mul(const CholJob* __restrict__ jobs, int s, int phase) {
    const CholJob& J = jobs[blockIdx.z];
    const int kp = J.kp;
    const int p = static_cast<int>(blockIdx.y);
    const int i0 = 2 * p * s, i1 = i0 + s;
    if (i1 >= J.kc || i1 + s > kp) return;
    const int tps = (s + CT - 1) / CT;
    const int tile = static_cast<int>(blockIdx.x);
    if (tile >= tps * tps) return;
    const int r0 = (tile / tps) * CT, q0 = (tile % tps) * CT;
    const double* A;
    const double* Bm;
    int64_t lda = kp, ldb;
    double* C;
    int64_t ldc;
    double alpha;
    double* T = J.T + static_cast<int64_t>(p) * s * s;
    if (phase == 0) {
        A = J.B + static_cast<int64_t>(i1) * kp + i0;
        Bm = J.Linv + static_cast<int64_t>(i0) * kp + i0;
        ldb = kp;
        C = T;
        ldc = s;
        alpha = 1.0;
    } else {
        A = J.Linv + static_cast<int64_t>(i1) * kp + i1;
        Bm = T;
        ldb = s;
        C = J.Linv + static_cast<int64_t>(i1) * kp + i0;
        ldc = kp;
        alpha = -1.0;
    }
    __shared__ double As[16][CT + 1];
    __shared__ double Bs[16][CT + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < s; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * CT; e += 256) {
            const int kk = e % 16, ii = e / 16;
            const int r = r0 + ii, k = k0 + kk;
            As[kk][ii] = (r < s && k < s) ? A[r * lda + k] : 0.0;
            const int kb = k0 + e / CT, jj = e % CT, c = q0 + jj;
            Bs[e / CT][jj] = (kb < s && c < s) ? Bm[kb * ldb + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[kk][ty * 4 + u];
                b[u] = Bs[kk][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = r0 + ty * 4 + u;
        if (r >= s) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = q0 + tx * 4 + v;
            if (c < s) C[r * ldc + c] = alpha * acc[u][v];
        }
    }
}

void launch_chol_inverse(const CholJob* jobs, int njobs, int max_kc, int max_kp, hipStream_t st) {
    if (njobs <= 0 || max_kc <= 0) return;
    const unsigned nj = static_cast<unsigned>(njobs);
    hipLaunchKernelGGL(k_chol_diag, dim3(static_cast<unsigned>((max_kc + 255) / 256), nj), dim3(256), 0, st, jobs);
    for (int c0 = 0; c0 < max_kc; c0 += CP) {
        const int below = max_kc - c0 - CP;
        const unsigned chunks = static_cast<unsigned>(below > 0 ? (below + 255) / 256 : 1);
        hipLaunchKernelGGL(k_chol_panel, dim3(chunks, nj), dim3(256), 0, st, jobs, c0);
        if (below > 0) {
            const int nt = (below + CT - 1) / CT;
            hipLaunchKernelGGL(k_chol_update, dim3(static_cast<unsigned>(nt * (nt + 1) / 2), nj), dim3(256), 0, st,
                               jobs, c0);
        }
    }
    hipLaunchKernelGGL(k_trinv_diag, dim3(static_cast<unsigned>(max_kp / CP), nj), dim3(64), 0, st, jobs);
    for (int s = CP; s < max_kp; s *= 2) {
        const int tps = (s + CT - 1) / CT;
        const unsigned pairs = static_cast<unsigned>(max_kp / (2 * s));
        for (int phase = 0; phase < 2; ++phase)
            hipLaunchKernelGGL(k_trinv_mul, dim3(static_cast<unsigned>(tps * tps), pairs, nj), dim3(256), 0, st, jobs,
                               s, phase);
    }
}

// Residual of the final eigenpairs: column i of R = G V (q x t row-major) against
// lam_i V[:, i]; the job is marked when ||r_i|| > tol * lam_0, or lam_i is not finite.
// One workgroup per 64 columns, lane = column, the four waves splitting the rows.
__global__ __launch_bounds__(256) void k_sub_residual(const double* __restrict__ R, const double* __restrict__ V,
                                                      const double* __restrict__ lam, int64_t q, int64_t t,
                                                      double tol, int* __restrict__ flag) {
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    __shared__ double part[4][64];
    double s = 0.0;
    if (c < t) {
        const double l = lam[c];
        for (int64_t r = w; r < q; r += 4) {
            const double d = R[r * t + c] - l * V[r * t + c];
            s += d * d;
        }
    }
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && c < t) {
        const double tot = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
        const double l0 = lam[0], l = lam[c];
        if (!(sqrt(tot) <= tol * l0) || !(l == l)) atomicOr(flag, 1);
    }
}

void launch_sub_residual(const double* R, const double* V, const double* lam, int64_t q, int64_t t, double tol,
                         int* flag, hipStream_t st) {
    if (q <= 0 || t <= 0) return;
    hipLaunchKernelGGL(k_sub_residual, dim3(static_cast<unsigned>((t + 63) / 64)), dim3(256), 0, st, R, V, lam, q,
                       t, tol, flag);
}

// H = (H + H^T) / 2 in place (k x k row-major)
__global__ void k_symmetrize(double* __restrict__ H, int64_t k) {
    const int64_t n = k * k;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t i = e / k, j = e % k;
        if (j < i) {
            const double v = 0.5 * (H[i * k + j] + H[j * k + i]);
            H[i * k + j] = v;
            H[j * k + i] = v;
        }
    }
}

void launch_symmetrize(double* H, int64_t k, hipStream_t st) {
    if (k <= 1) return;
    hipLaunchKernelGGL(k_symmetrize, dim3(static_cast<unsigned>(std::min<int64_t>((k * k + 255) / 256, 4096))),
                       dim3(256), 0, st, H, k);
}

}  // namespace fastpi

namespace fastpi {

// p[i * ld + i] = v for i in [i0, i1)
__global__ void k_fill_diag(double* __restrict__ p, int64_t ld, int64_t i0, int64_t i1, double v) {
    for (int64_t i = i0 + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < i1;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i * ld + i] = v;
}

void launch_fill_diag(double* p, int64_t ld, int64_t i0, int64_t i1, double v, hipStream_t st) {
    if (i1 <= i0) return;
    hipLaunchKernelGGL(k_fill_diag, dim3(static_cast<unsigned>(std::min<int64_t>((i1 - i0 + 255) / 256, 1024))),
                       dim3(256), 0, st, p, ld, i0, i1, v);
}

}  // namespace fastpi
