// Preconditioner of the core eigensolver: Cholesky factorisation with diagonal pivoting of
// the positive semidefinite core G, G = R^T R, computed in the original index order (row j
// of R is the j-th pivot step; its entries at indices pivoted earlier are zero). One-sided
// Jacobi then runs on the columns of X = R^T instead of on G: R^T R = G, so the columns
// converge to u_c sqrt(lambda_c) with u_c the eigenvectors of G, and lambda_c = ||x_c||^2.
// Pivoting on the largest remaining diagonal makes R strongly graded and R^T close to
// orthogonal columns scaled by the pivots, so far fewer Jacobi sweeps are needed than on G
// itself (the pivoted-QR preconditioning of one-sided Jacobi, applied through the Gram
// matrix). The factorisation stops when the largest remaining diagonal falls below
// (ld eps)^2 of the largest initial one; the columns past that point stay zero and the
// neglected trailing part is far below the rounding level of G.
//
// Blocked by panels of pivot steps: one workgroup per job factors a panel (each step:
// arg-max of the remaining diagonal, then the new column from the trailing matrix minus the
// panel's earlier columns), and a tiled kernel subtracts the panel's outer product from the
// trailing matrix. Every thread owns fixed rows (i = tid + k * PT), so it only re-reads
// global values it wrote itself; the only cross-thread data (the pivot and the pivot row's
// panel entries) goes through LDS.
#include <cfloat>

#include "device_common.h"
#include "kernels.h"

namespace fastpi {

constexpr int PT = 1024;    // threads of the panel kernel
constexpr int UT = 64;      // trailing-update tile

// X = 0 and the working copy A of G for the jobs that take the start; X = G (and the
// factorisation marked done) for the others of the set.
__global__ void k_pchol_init(const EigJob* __restrict__ jobs, int* __restrict__ pstate) {
    const int jb = blockIdx.y;
    const EigJob& J = jobs[jb];
    const int64_t q = J.q, ld = J.ld;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (!J.squared) {
        for (int64_t e = t0; e < ld * ld; e += stride) {
            const int64_t r = e % ld, c = e / ld;
            J.X[e] = (r < q && c < q) ? J.G[r * q + c] : 0.0;
        }
        if (t0 == 0) {
            pstate[2 * jb] = 0;
            pstate[2 * jb + 1] = 1;
        }
        return;
    }
    for (int64_t e = t0; e < ld * ld; e += stride) J.X[e] = 0.0;
    if (J.A != J.G)
        for (int64_t e = t0; e < q * q; e += stride) J.A[e] = J.G[e];
    double* d = J.Hpart;
    for (int64_t i = t0; i < q; i += stride) d[i] = J.G[i * q + i];
    if (t0 == 0) {
        pstate[2 * jb] = 0;
        pstate[2 * jb + 1] = 0;
    }
}

// (value, index) arg-max with ties to the lower index
__device__ __forceinline__ void better(double& v, int& i, double ov, int oi) {
    if (ov > v || (ov == v && oi < i)) {
        v = ov;
        i = oi;
    }
}

// A -= X[:, j0:j0+P] X[:, j0:j0+P]^T over the job's q x q trailing matrix (64 x 64 tiles).
// Skipped once the factorisation is done (no later panel reads A).
template <int P>
__global__ __launch_bounds__(256) void k_pchol_update(const EigJob* __restrict__ jobs,
                                                      const int* __restrict__ pstate, int j0) {
    const int jb = blockIdx.y;
    const EigJob& J = jobs[jb];
    const int64_t q = J.q;
    if (j0 >= q || pstate[2 * jb + 1]) return;
    const int tiles = static_cast<int>((q + UT - 1) / UT);
    if (static_cast<int>(blockIdx.x) >= tiles * tiles) return;
    const int64_t i0 = static_cast<int64_t>(blockIdx.x % tiles) * UT;
    const int64_t c0 = static_cast<int64_t>(blockIdx.x / tiles) * UT;
    const int64_t ld = J.ld;
    const double* X = J.X;
    __shared__ double Xi[P][UT + 1];
    __shared__ double Xc[P][UT + 1];
    for (int e = threadIdx.x; e < P * UT; e += 256) {
        const int l = e / UT, t = e % UT;
        Xi[l][t] = (i0 + t < q) ? X[i0 + t + ld * (j0 + l)] : 0.0;
        Xc[l][t] = (c0 + t < q) ? X[c0 + t + ld * (j0 + l)] : 0.0;
    }
    __syncthreads();
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4] = {};
#pragma unroll 4
    for (int l = 0; l < P; ++l) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = Xi[l][tx + 16 * u];
            b[u] = Xc[l][ty * 4 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    // A is symmetric and addressed as A[i + q c]; consecutive threads take consecutive i
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t c = c0 + ty * 4 + v;
        if (c >= q) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + tx + 16 * u;
            if (i < q) J.A[i + q * c] -= acc[u][v];
        }
    }
}

// Register-resident panel: thread t owns rows t + PT u (u < R) and keeps their remaining
// diagonal and their entries in the panel's columns in registers, so a pivot step reads
// only the pivot column of A from memory. Two barriers per step.
template <int R, int P>
__global__ __launch_bounds__(PT) void k_pchol_panel_reg(const EigJob* __restrict__ jobs,
                                                        int* __restrict__ pstate, int j0) {
    const int jb = blockIdx.x;
    const EigJob& J = jobs[jb];
    const int q = static_cast<int>(J.q);
    if (j0 >= q || pstate[2 * jb + 1]) return;
    const int64_t ld = J.ld;
    double* X = J.X;
    const double* A = J.A;
    double* d = J.Hpart;
    __shared__ double s_v[PT / kWave];
    __shared__ int s_i[PT / kWave];
    __shared__ double s_piv[P];
    __shared__ double s_floor;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    double dr[R], xr[R][P];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int i = threadIdx.x + u * PT;
        dr[u] = i < q ? d[i] : -DBL_MAX;
#pragma unroll
        for (int l = 0; l < P; ++l) xr[u][l] = 0.0;
    }
    if (j0 == 0) {
        // stop threshold from the largest initial diagonal
        double mx = 0.0;
#pragma unroll
        for (int u = 0; u < R; ++u) mx = dr[u] > mx ? dr[u] : mx;
        mx = wave_max(mx);
        if (lane == 0) s_v[wave] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = 0.0;
            for (int w = 0; w < PT / kWave; ++w) m = s_v[w] > m ? s_v[w] : m;
            const double e = static_cast<double>(ld) * DBL_EPSILON;
            J.lam[ld + 1] = e * e * m;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) s_floor = J.lam[ld + 1];
    const int j1 = min(q, j0 + P);
    for (int j = j0; j < j1; ++j) {
        const int jj = j - j0;
        double bv = -DBL_MAX;
        int bi = q;
#pragma unroll
        for (int u = 0; u < R; ++u) better(bv, bi, dr[u], threadIdx.x + u * PT);
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off, kWave);
            const int oi = __shfl_xor(bi, off, kWave);
            better(bv, bi, ov, oi);
        }
        if (lane == 0) {
            s_v[wave] = bv;
            s_i[wave] = bi;
        }
        __syncthreads();
        // every wave reduces the wave results: one per lane, then a butterfly
        double dp = lane < PT / kWave ? s_v[lane] : -DBL_MAX;
        int p = lane < PT / kWave ? s_i[lane] : q;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double ov = __shfl_xor(dp, off, kWave);
            const int oi = __shfl_xor(p, off, kWave);
            better(dp, p, ov, oi);
        }
        if (!(dp > s_floor) || p >= q) {
            if (threadIdx.x == 0) {
                pstate[2 * jb] = j;       // rank found
                pstate[2 * jb + 1] = 1;   // done
            }
            return;
        }
        if (threadIdx.x == p % PT) {
            const int up = p / PT;
#pragma unroll
            for (int l = 0; l < P; ++l) {
                double v = 0.0;
#pragma unroll
                for (int u = 0; u < R; ++u)
                    if (u == up) v = xr[u][l];
                s_piv[l] = l < jj ? v : 0.0;
            }
        }
        // after this barrier every thread has read s_v and s_i; the next writes of s_v,
        // s_i and s_piv come after the next step's first barrier, which every reader of
        // this step's s_piv has passed
        __syncthreads();
        const double r = sqrt(dp);
        const double rinv = 1.0 / r;
        const double* Ap = A + static_cast<int64_t>(p) * q;   // column p of the symmetric A
        double av[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int i = threadIdx.x + u * PT;
            av[u] = i < q ? Ap[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int i = threadIdx.x + u * PT;
            if (i >= q) continue;
            double x;
            if (i == p) {
                x = r;
                dr[u] = -DBL_MAX;
            } else if (dr[u] == -DBL_MAX) {
                x = 0.0;
            } else {
                double sacc = av[u];
#pragma unroll
                for (int l = 0; l < P; ++l) sacc -= xr[u][l] * s_piv[l];
                x = sacc * rinv;
                dr[u] -= x * x;
            }
#pragma unroll
            for (int l = 0; l < P; ++l)
                if (l == jj) xr[u][l] = x;
            X[i + ld * j] = x;
        }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int i = threadIdx.x + u * PT;
        if (i < q) d[i] = dr[u];
    }
    if (threadIdx.x == 0) {
        pstate[2 * jb] = j1;
        if (j1 >= q) pstate[2 * jb + 1] = 1;
    }
}

// Panel for cores above the register variants' reach: the rows' remaining diagonal and
// panel entries stay in global memory, each thread re-reading only its own rows (which it
// wrote); the loads of RG rows are issued together.
constexpr int PG = 16;   // panel width of this variant
template <int RG>
__global__ __launch_bounds__(PT) void k_pchol_panel_glob(const EigJob* __restrict__ jobs,
                                                         int* __restrict__ pstate, int j0) {
    const int jb = blockIdx.x;
    const EigJob& J = jobs[jb];
    const int q = static_cast<int>(J.q);
    if (j0 >= q || pstate[2 * jb + 1]) return;
    const int64_t ld = J.ld;
    double* X = J.X;
    const double* A = J.A;
    double* d = J.Hpart;
    __shared__ double s_v[PT / kWave];
    __shared__ int s_i[PT / kWave];
    __shared__ double s_piv[PG];
    __shared__ double s_floor;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    if (j0 == 0) {
        double mx = 0.0;
        for (int i = threadIdx.x; i < q; i += PT) mx = d[i] > mx ? d[i] : mx;
        mx = wave_max(mx);
        if (lane == 0) s_v[wave] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = 0.0;
            for (int w = 0; w < PT / kWave; ++w) m = s_v[w] > m ? s_v[w] : m;
            const double e = static_cast<double>(ld) * DBL_EPSILON;
            J.lam[ld + 1] = e * e * m;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) s_floor = J.lam[ld + 1];
    const int j1 = min(q, j0 + PG);
    for (int j = j0; j < j1; ++j) {
        const int jj = j - j0;
        double bv = -DBL_MAX;
        int bi = q;
        for (int base = 0; base < q; base += RG * PT) {
            double dv[RG];
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                const int i = base + threadIdx.x + u * PT;
                dv[u] = i < q ? d[i] : -DBL_MAX;
            }
#pragma unroll
            for (int u = 0; u < RG; ++u) better(bv, bi, dv[u], base + threadIdx.x + u * PT);
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off, kWave);
            const int oi = __shfl_xor(bi, off, kWave);
            better(bv, bi, ov, oi);
        }
        if (lane == 0) {
            s_v[wave] = bv;
            s_i[wave] = bi;
        }
        __syncthreads();
        double dp = lane < PT / kWave ? s_v[lane] : -DBL_MAX;
        int p = lane < PT / kWave ? s_i[lane] : q;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double ov = __shfl_xor(dp, off, kWave);
            const int oi = __shfl_xor(p, off, kWave);
            better(dp, p, ov, oi);
        }
        if (!(dp > s_floor) || p >= q) {
            if (threadIdx.x == 0) {
                pstate[2 * jb] = j;
                pstate[2 * jb + 1] = 1;
            }
            return;
        }
        if (threadIdx.x == p % PT) {
            double pv[PG];
#pragma unroll
            for (int l = 0; l < PG; ++l) pv[l] = l < jj ? X[p + ld * (j0 + l)] : 0.0;
#pragma unroll
            for (int l = 0; l < PG; ++l) s_piv[l] = pv[l];
        }
        // every thread has read s_v and s_i; the next writes of s_v, s_i and s_piv come after
        // the next step's first barrier, which every reader of this step's s_piv has passed
        __syncthreads();
        const double r = sqrt(dp);
        const double rinv = 1.0 / r;
        const double* Ap = A + static_cast<int64_t>(p) * q;
        for (int base = 0; base < q; base += RG * PT) {
            double av[RG], dv[RG], xv[RG][PG];
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                const int i = base + threadIdx.x + u * PT;
                const bool in = i < q;
                av[u] = in ? Ap[i] : 0.0;
                dv[u] = in ? d[i] : -DBL_MAX;
#pragma unroll
                for (int l = 0; l < PG; ++l) xv[u][l] = (in && l < jj) ? X[i + ld * (j0 + l)] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < RG; ++u) {
                const int i = base + threadIdx.x + u * PT;
                if (i >= q) continue;
                double x;
                if (i == p) {
                    x = r;
                    d[i] = -DBL_MAX;
                } else if (dv[u] == -DBL_MAX) {
                    x = 0.0;
                } else {
                    double sacc = av[u];
#pragma unroll
                    for (int l = 0; l < PG; ++l) sacc -= xv[u][l] * s_piv[l];
                    x = sacc * rinv;
                    d[i] = dv[u] - x * x;
                }
                X[i + ld * j] = x;
            }
        }
    }
    if (threadIdx.x == 0) {
        pstate[2 * jb] = j1;
        if (j1 >= q) pstate[2 * jb + 1] = 1;
    }
}

template <int R, int P>
static void run_panels(const EigSet& es, unsigned nj, unsigned tgrid, hipStream_t st) {
    const int panels = static_cast<int>((es.max_q + P - 1) / P);
    for (int pnl = 0; pnl < panels; ++pnl) {
        const int j0 = pnl * P;
        hipLaunchKernelGGL((k_pchol_panel_reg<R, P>), dim3(nj), dim3(PT), 0, st, es.jobs, es.pstate, j0);
        if (pnl + 1 < panels)
            hipLaunchKernelGGL(k_pchol_update<P>, dim3(tgrid, nj), dim3(256), 0, st, es.jobs, es.pstate, j0);
    }
}

void pchol_run(const EigSet& es, hipStream_t st) {
    if (es.njobs == 0) return;
    const unsigned nj = static_cast<unsigned>(es.njobs);
    const unsigned gx = static_cast<unsigned>(std::min<int64_t>((es.max_ld * es.max_ld + 255) / 256, 4096));
    hipLaunchKernelGGL(k_pchol_init, dim3(gx, nj), dim3(256), 0, st, es.jobs, es.pstate);
    const int64_t tiles = (es.max_q + UT - 1) / UT;
    const unsigned tgrid = static_cast<unsigned>(tiles * tiles);
    // rows per thread R and panel width P with R * P <= 32 register doubles (16 at R = 8)
    if (es.max_q <= PT) {
        run_panels<1, 16>(es, nj, tgrid, st);
    } else if (es.max_q <= 2 * PT) {
        run_panels<2, 16>(es, nj, tgrid, st);
    } else if (es.max_q <= 4 * PT) {
        run_panels<4, 8>(es, nj, tgrid, st);
    } else if (es.max_q <= 8 * PT) {
        run_panels<8, 2>(es, nj, tgrid, st);
    } else {
        const int panels = static_cast<int>((es.max_q + PG - 1) / PG);
        for (int pnl = 0; pnl < panels; ++pnl) {
            const int j0 = pnl * PG;
            hipLaunchKernelGGL(k_pchol_panel_glob<2>, dim3(nj), dim3(PT), 0, st, es.jobs, es.pstate, j0);
            if (pnl + 1 < panels)
                hipLaunchKernelGGL(k_pchol_update<PG>, dim3(tgrid, nj), dim3(256), 0, st, es.jobs, es.pstate, j0);
        }
    }
}

}  // namespace fastpi
