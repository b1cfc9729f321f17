// Dense kernels of the subspace core solver (the top-t eigenpairs of an update's Gram
// matrix G by subspace iteration, Rayleigh-Ritz on the converged basis): the Cholesky QR
// that orthonormalises the iterate (B = Y^T Y = L L^T, Q = Y L^-T) and the residual check of
// the final eigenpairs. Everything is batched over the cores of one update step ("jobs"):
// one launch per kernel and panel for all of them.
//
// Cholesky with the inverse accumulated on the way (B kp x kp row-major, kp = k rounded up
// to 64, the identity past k): right-looking over panels of 64 columns, two launches each.
//  * k_cq_panel(p): every workgroup loads the 64 x 64 diagonal block, factors it and inverts
//    the factor in LDS, X = L_pp^-1 (blocked by 16); then its 64 x 64 tile: rows below the
//    panel, L21 = B21 X^T (in place in B), or columns of block row p of M = L^-1,
//    M_pj = -X W_pj (j < p), where W_pj = sum_{l<p} L_pl M_lj was accumulated in M's own
//    storage; workgroup 0 writes M_pp = X.
//  * k_cq_update(p): the trailing lower triangle of B minus L21 L21^T, and W_ij += L_ip M_pj
//    for every block row i > p and column block j <= p (the first term, j = p, assigned).
// A pivot whose square falls to kp * eps of its column's original diagonal marks the job
// (the block lost rank numerically); the caller then takes the Jacobi route instead. M's
// upper triangle stays zero, so Q = Y M^T is one GEMM.
#include <cfloat>

#include "device_common.h"
#include "kernels.h"

namespace fastpi {

constexpr int CP = 64;    // panel width (= the wave width of the diagonal factorisation)
constexpr int CT = 64;    // tile of the trailing products

// rocPRIM's wave-level barrier: orders LDS accesses of one wave without a workgroup barrier
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// original diagonal of every job's B (the reference of the rank test)
__global__ void k_chol_diag(const CholJob* __restrict__ jobs) {
    const CholJob& J = jobs[blockIdx.y];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < J.kp; i += gridDim.x * blockDim.x)
        J.dg[i] = J.B[static_cast<int64_t>(i) * J.kp + i];
}

__device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), lane);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// The panel's diagonal block D (64 x 64, in LDS) factored in place, L lower, and X = L^-1,
// blocked by 16. For each 16-block: wave 0 holds the block's 16 rows in registers (lane i:
// row i) and factors it column by column: the pivot comes to every lane by readlane, its
// reciprocal square root from the hardware estimate refined to FP64, and each new column of
// L goes to the other lanes through a 16 x 16 LDS buffer (one write, broadcast reads, no
// workgroup barrier). It then inverts the 16 x 16 factor in registers (lane j: column j of the
// inverse, L read back from that buffer) and writes both. All waves then form the rows below,
// L_ib = D_ib X_bb^T (independent dot products), and update the rest of D. The block rows of
// X below the diagonal follow at the end. Returns the number of pivots that lost rank.
__device__ int cq_factor_invert(double (*D)[CP + 1], double (*X)[CP + 1], double (*T)[CP + 1], const double* dg,
                                double lim) {
    const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
    __shared__ int nbad;
    __shared__ double lims[CP];   // rank-test threshold of every pivot
    __shared__ double Lc[16][16];  // Lc[c][i] = L_ic of the 16-block being factored
    if (tid == 0) nbad = 0;
    if (tid < CP) lims[tid] = lim * dg[tid];
    for (int e = tid; e < CP * CP; e += 256) X[e / CP][e % CP] = 0.0;
    __syncthreads();
    // wave 0: factor the 16-block at bb and invert its factor (L into D, X_bb into X)
    auto factor16 = [&](int bb) __attribute__((always_inline)) {
        const int li = lane < 16 ? lane : 15;
        double r[16];
#pragma unroll
        for (int l = 0; l < 16; ++l) r[l] = D[bb + li][bb + l];
        double dv[16];   // 1 / L[c][c] (the same on every lane)
        int lost_here = 0;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const double sc = lane_value(r[c], c);   // the same on every lane: uniform branches
            const bool lost = !(sc > lims[bb + c]);
            lost_here += lost ? 1 : 0;
            double piv = 1.0, rp = 1.0;   // a lost pivot keeps the arithmetic finite
            if (!lost) {
                if (sc > 1e-290 && sc < 1e290) {
                    rp = rsq3(sc);
                    piv = sc * rp;
                } else {
                    piv = sqrt(sc);
                    rp = 1.0 / piv;
                }
            }
            dv[c] = rp;
            const double l = lane > c ? r[c] * rp : (lane == c ? piv : 0.0);
            r[c] = l;
            if (lane < 16) Lc[c][lane] = l;
            wave_sync();
#pragma unroll
            for (int j = c + 1; j < 16; ++j) r[j] -= l * Lc[c][j];
        }
        // column `lane` of the inverse: x_i = -(sum_{l<i} L_il x_l) / L_ii, x_lane = 1 / L_ll
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            double v = 0.0;
#pragma unroll
            for (int l = 0; l < i; ++l) v += Lc[l][i] * x[l];
            x[i] = i < lane ? 0.0 : (i == lane ? dv[i] : -v * dv[i]);
        }
        if (lane < 16) {
#pragma unroll
            for (int l = 0; l < 16; ++l) {
                if (l <= lane) D[bb + lane][bb + l] = r[l];
                X[bb + l][bb + lane] = x[l];
            }
        }
        if (lane == 0 && lost_here) nbad += lost_here;
    };
    // step bb: the rows below the factored block, the next diagonal block's update, then (with
    // one step of lookahead) wave 0 factors the next block while the other waves update the
    // rest of the trailing part, which that factorisation does not touch; the first step only
    // factors the first block
#pragma unroll 1
    for (int bb = -16; bb + 16 < CP; bb += 16) {
        const int nr = CP - bb - 16;   // rows below the 16-block at bb
        if (bb >= 0) {
            // rows below: L_ib = D_ib X_bb^T, X_bb lower triangular
            double v3[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int e = tid + 256 * u;
                v3[u] = 0.0;
                if (e < nr * 16) {
                    const int i = bb + 16 + e / 16, j = e % 16;
#pragma unroll
                    for (int l = 0; l < 16; ++l)
                        if (l <= j) v3[u] += D[i][bb + l] * X[bb + j][bb + l];
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int e = tid + 256 * u;
                if (e < nr * 16) D[bb + 16 + e / 16][bb + e % 16] = v3[u];
            }
            __syncthreads();
            // the next diagonal block, rows and columns [bb + 16, bb + 32), minus L L^T
            const int i = bb + 16 + tid / 16, j = bb + 16 + tid % 16;
            if (j <= i) {
                double v = 0.0;
#pragma unroll
                for (int l = 0; l < 16; ++l) v += D[i][bb + l] * D[j][bb + l];
                D[i][j] -= v;
            }
            __syncthreads();
        }
        if (w == 0) {
            factor16(bb + 16);
        } else if (bb >= 0) {
            // rows [bb + 32, CP) of the trailing lower triangle
            const int nr2 = nr - 16;
            for (int e = tid - 64; e < nr2 * nr; e += 192) {
                const int i = bb + 32 + e / nr, j = bb + 16 + e % nr;
                if (j > i) continue;
                double v = 0.0;
#pragma unroll
                for (int l = 0; l < 16; ++l) v += D[i][bb + l] * D[j][bb + l];
                D[i][j] -= v;
            }
        }
        __syncthreads();
    }
    // block row bi: T_j = sum_{l=j}^{bi-1} L_{bi,l} X_{l,j}, then X_{bi,j} = -X_{bi,bi} T_j (j < bi).
    // X is zero above its diagonal blocks (cleared above, and the diagonal blocks are written
    // with their zeros), so each sum runs over all rows of the earlier blocks with no
    // predicates; four partial sums keep the LDS loads and the FMAs of a thread independent
#pragma unroll
    for (int bi = 1; bi < 4; ++bi) {
        const int r0 = bi * 16, n = bi * 16;   // columns [0, n) of block row bi
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int e = tid + 256 * u;
            if (e < 16 * n) {
                const int rr = e / n, cc = e % n;
                double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int l = 0; l < r0; ++l) v[l & 3] += D[r0 + rr][l] * X[l][cc];
                T[rr][cc] = (v[0] + v[1]) + (v[2] + v[3]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int e = tid + 256 * u;
            if (e < 16 * n) {
                const int rr = e / n, cc = e % n;
                double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int l = 0; l < 16; ++l) v[l & 3] += X[r0 + rr][r0 + l] * T[l][cc];
                X[r0 + rr][cc] = -((v[0] + v[1]) + (v[2] + v[3]));
            }
        }
        __syncthreads();
    }
    return nbad;
}

__global__ __launch_bounds__(256) void k_cq_panel(const CholJob* __restrict__ jobs, int c0) {
    const CholJob& J = jobs[blockIdx.y];
    const int kp = J.kp;
    if (c0 >= kp) return;
    const int c1 = c0 + CP;
    const int nrt = (kp - c1) / CT;   // row tiles of L21
    const int nct = c0 / CT;          // column tiles of M's block row p
    const int tile = static_cast<int>(blockIdx.x);
    if (tile > 0 && tile >= nrt + nct) return;
    __shared__ double D[CP][CP + 1];
    __shared__ double X[CP][CP + 1];
    __shared__ double S[CP][CT + 1];
    const int tid = threadIdx.x;
    double* B = J.B;
    double* M = J.M;
    {
        // every thread's 16 loads in flight before the first store to LDS
        double v[CP * CP / 256];
#pragma unroll
        for (int u = 0; u < CP * CP / 256; ++u) {
            const int e = tid + 256 * u;
            v[u] = B[static_cast<int64_t>(c0 + e / CP) * kp + c0 + e % CP];
        }
#pragma unroll
        for (int u = 0; u < CP * CP / 256; ++u) {
            const int e = tid + 256 * u;
            D[e / CP][e % CP] = v[u];
        }
    }
    __syncthreads();
    const int bad = cq_factor_invert(D, X, S, J.dg + c0, static_cast<double>(kp) * DBL_EPSILON);
    if (tile == 0) {
        for (int e = tid; e < CP * CP; e += 256) {
            const int i = e / CP, j = e % CP;
            M[static_cast<int64_t>(c0 + i) * kp + c0 + j] = X[i][j];
        }
        if (tid == 0 && bad) atomicOr(J.flag, 1);
    }
    if (tile >= nrt + nct) return;
    const int tx = tid % 16, ty = tid / 16;
    double acc[4][4] = {};
    if (tile < nrt) {
        // rows [r0, r0 + 64) of L21 = A21 X^T
        const int r0 = c1 + tile * CT;
        double v[CT * CP / 256];
#pragma unroll
        for (int u = 0; u < CT * CP / 256; ++u) {
            const int e = tid + 256 * u;
            v[u] = B[static_cast<int64_t>(r0 + e / CP) * kp + c0 + e % CP];
        }
#pragma unroll
        for (int u = 0; u < CT * CP / 256; ++u) {
            const int e = tid + 256 * u;
            S[e % CP][e / CP] = v[u];
        }
        __syncthreads();
#pragma unroll 8
        for (int l = 0; l < CP; ++l) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = S[l][ty * 4 + u];
                b[u] = X[tx * 4 + u][l];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                B[static_cast<int64_t>(r0 + ty * 4 + u) * kp + c0 + tx * 4 + v] = acc[u][v];
    } else {
        // columns [q0, q0 + 64) of M's block row p: M_pj = -X W_pj
        const int q0 = (tile - nrt) * CT;
        double v[CP * CT / 256];
#pragma unroll
        for (int u = 0; u < CP * CT / 256; ++u) {
            const int e = tid + 256 * u;
            v[u] = M[static_cast<int64_t>(c0 + e / CT) * kp + q0 + e % CT];
        }
#pragma unroll
        for (int u = 0; u < CP * CT / 256; ++u) {
            const int e = tid + 256 * u;
            S[e / CT][e % CT] = v[u];
        }
        __syncthreads();
#pragma unroll 8
        for (int l = 0; l < CP; ++l) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = X[ty * 4 + u][l];
                b[u] = S[l][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                M[static_cast<int64_t>(c0 + ty * 4 + u) * kp + q0 + tx * 4 + v] = -acc[u][v];
    }
}

// After panel p: B[i][j] -= sum_l L[i][c0+l] L[j][c0+l] on the lower triangle of
// [c1, kp)^2 (tiles numbered row by row), then W tiles: M[i][j] (+)= sum_l L[i][c0+l]
// M[c0+l][j] for rows [c1, kp) and columns [0, c1) (assigned in columns [c0, c1)).
__global__ __launch_bounds__(256) void k_cq_update(const CholJob* __restrict__ jobs, int c0) {
    const CholJob& J = jobs[blockIdx.y];
    const int kp = J.kp;
    const int c1 = c0 + CP;
    if (c1 >= kp) return;
    const int nt = (kp - c1) / CT;                   // kp - c1 is a multiple of 64
    const int ntri = nt * (nt + 1) / 2;
    const int nw = nt * (c1 / CT);
    int tile = static_cast<int>(blockIdx.x);
    if (tile >= ntri + nw) return;
    __shared__ double Ls[CP][CT + 1];   // L rows of the output tile's rows, transposed
    __shared__ double Rs[CP][CT + 1];   // the right operand: L rows (B part) or M block row p
    int i0, j0;
    bool wpart = tile >= ntri;
    double* B = J.B;
    double* M = J.M;
    if (!wpart) {
        int ti = static_cast<int>((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
        while (ti * (ti + 1) / 2 > tile) --ti;
        const int tj = tile - ti * (ti + 1) / 2;
        i0 = c1 + ti * CT;
        j0 = c1 + tj * CT;
    } else {
        tile -= ntri;
        const int ncw = c1 / CT;
        i0 = c1 + (tile / ncw) * CT;
        j0 = (tile % ncw) * CT;
    }
    {
        // every thread's loads in flight before the first store to LDS
        constexpr int NU = CP * CT / 256;
        double a[NU], bv[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int e = threadIdx.x + 256 * u;
            a[u] = B[static_cast<int64_t>(i0 + e / CP) * kp + c0 + e % CP];
            bv[u] = wpart ? M[static_cast<int64_t>(c0 + e / CT) * kp + j0 + e % CT]
                          : B[static_cast<int64_t>(j0 + e / CP) * kp + c0 + e % CP];
        }
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int e = threadIdx.x + 256 * u;
            Ls[e % CP][e / CP] = a[u];
            if (wpart) Rs[e / CT][e % CT] = bv[u];
            else Rs[e % CP][e / CP] = bv[u];
        }
    }
    __syncthreads();
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4] = {};
#pragma unroll 8
    for (int l = 0; l < CP; ++l) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = Ls[l][ty * 4 + u];
            b[u] = Rs[l][tx * 4 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    if (!wpart) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + ty * 4 + u;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = j0 + tx * 4 + v;
                if (j <= i) B[static_cast<int64_t>(i) * kp + j] -= acc[u][v];
            }
        }
    } else {
        const bool first = j0 >= c0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + ty * 4 + u;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = j0 + tx * 4 + v;
                double* o = M + static_cast<int64_t>(i) * kp + j;
                *o = first ? acc[u][v] : *o + acc[u][v];
            }
        }
    }
}

void launch_chol_inverse(const CholJob* jobs, int njobs, int max_kp, hipStream_t st, KernelTimer* timer) {
    if (njobs <= 0 || max_kp <= 0) return;
    const unsigned nj = static_cast<unsigned>(njobs);
    hipLaunchKernelGGL(k_chol_diag, dim3(static_cast<unsigned>((max_kp + 255) / 256), nj), dim3(256), 0, st, jobs);
    for (int c0 = 0; c0 < max_kp; c0 += CP) {
        const int c1 = c0 + CP;
        const unsigned tiles = static_cast<unsigned>(std::max(1, (max_kp - c1) / CT + c0 / CT));
        FASTPI_LAUNCH(timer, KT_CQ_PANEL, k_cq_panel, dim3(tiles, nj), dim3(256), 0, st, jobs, c0);
        if (c1 < max_kp) {
            const int nt = (max_kp - c1) / CT;
            const unsigned tiles = static_cast<unsigned>(nt * (nt + 1) / 2 + nt * (c1 / CT));
            hipLaunchKernelGGL(k_cq_update, dim3(tiles, nj), dim3(256), 0, st, jobs, c0);
        }
    }
}

// Residual of the final eigenpairs: column i of R = G V (q x t row-major) against
// lam_i V[:, i]; the job is marked when ||r_i|| > tol * lam_0, or lam_i is not finite.
// One workgroup per 64 columns, lane = column, sixteen waves splitting the rows.
constexpr int RES_WAVES = 16;
__global__ __launch_bounds__(RES_WAVES * 64) void k_sub_residual(const double* __restrict__ R,
                                                                const double* __restrict__ V,
                                                                const double* __restrict__ lam, int64_t q, int64_t t,
                                                                double tol, int* __restrict__ flag) {
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    __shared__ double part[RES_WAVES][64];
    // wave w sums rows w, w + RES_WAVES, ... of column c, four rows' loads in flight at once
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (c < t) {
        const double l = lam[c];
        int64_t r = w;
        for (; r + 3 * RES_WAVES < q; r += 4 * RES_WAVES) {
            double x[4], y[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                x[u] = R[(r + u * RES_WAVES) * t + c];
                y[u] = V[(r + u * RES_WAVES) * t + c];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double d = x[u] - l * y[u];
                s[u] += d * d;
            }
        }
        for (; r < q; r += RES_WAVES) {
            const double d = R[r * t + c] - l * V[r * t + c];
            s[0] += d * d;
        }
    }
    part[w][lane] = (s[0] + s[1]) + (s[2] + s[3]);
    __syncthreads();
    if (w == 0 && c < t) {
        double tot = 0.0;
#pragma unroll
        for (int k = 0; k < RES_WAVES; ++k) tot += part[k][lane];
        const double l0 = lam[0], l = lam[c];
        if (!(sqrt(tot) <= tol * l0) || !(l == l)) atomicOr(flag, 1);
    }
}

void launch_sub_residual(const double* R, const double* V, const double* lam, int64_t q, int64_t t, double tol,
                         int* flag, hipStream_t st) {
    if (q <= 0 || t <= 0) return;
    hipLaunchKernelGGL(k_sub_residual, dim3(static_cast<unsigned>((t + 63) / 64)), dim3(RES_WAVES * 64), 0, st, R, V,
                       lam, q, t, tol, flag);
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
