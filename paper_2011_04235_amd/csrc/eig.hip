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

// Rotation of the symmetric 2x2 [[hpp, hpq], [hpq, hqq]] for the inner sweeps. The angle
// is only needed approximately (the outer sweeps continue until every pair is orthogonal),
// but c and s must form an exactly orthogonal pair: tan(theta) is taken in FP32 from the
// FP64 entries, then (c, s) is renormalised in FP64 with a Newton-corrected reciprocal
// square root so that c^2 + s^2 = 1 to FP64 rounding.
__device__ __forceinline__ void fast_rotation(double hpp, double hqq, double hpq, double& c, double& s) {
    c = 1.0;
    s = 0.0;
    const double ahpq = fabs(hpq);
    const double dd = hqq - hpp;
    // negligible coupling (also covers hpq == 0 and non-finite input)
    if (!(ahpq > 1e-17 * (fabs(hpp) + fabs(hqq)))) return;
    const double zeta64 = dd / (2.0 * hpq);
    const float zeta = static_cast<float>(zeta64);
    const float az = fabsf(zeta);
    float t;
    if (az > 1e15f || !(az == az)) {
        t = static_cast<float>(0.5 / zeta64);
    } else {
        t = 1.0f / (az + sqrtf(1.0f + zeta * zeta));
        if (zeta < 0) t = -t;
    }
    const double td = static_cast<double>(t);
    const double x = 1.0 + td * td;
    double y = static_cast<double>(rsqrtf(static_cast<float>(x)));
    y = y * (1.5 - 0.5 * x * y * y);
    y = y * (1.5 - 0.5 * x * y * y);
    c = y;
    s = y * td;
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

// One workgroup of PW * PW threads per pair, thread (i, j) owning H[i][j] and W[i][j] in
// registers. The partials are summed in chunk order; if the pair is not yet orthogonal
// to `tol`, `inner_sweeps` cyclic Jacobi sweeps (31 steps of 16 disjoint rotations) make
// H diagonal and W accumulates the rotations. In each step every wave derives the
// rotations of rows i and j itself from the shared copy of H, then thread (i, j) forms
// (J^T H J)[i][j] from H[i][j], H[i][j'], H[i'][j], H[i'][j'] and (W J)[i][j] from
// W[i][j], W[i][j'], writing into the other half of a double buffer: one barrier a step.
__global__ __launch_bounds__(PW * PW) void k_eig_solve(const double* __restrict__ Hpart, int nchunk,
                                                       const int2* __restrict__ pairs, int nblk,
                                                       double* __restrict__ Wout,
                                                       int* __restrict__ flag,
                                                       int* __restrict__ rot_count, double tol,
                                                       int inner_sweeps) {
    __shared__ double Hs[2][PW][PW + 1];
    __shared__ double Ws[2][PW][PW + 1];
    __shared__ int s_need;
    const int pair = blockIdx.x;
    const int2 pb = pairs[pair];
    if (pb.x >= nblk) {
        if (threadIdx.x == 0) flag[pair] = 0;
        return;
    }
    const int i = threadIdx.x / PW, j = threadIdx.x % PW;
    const double* Hp = Hpart + static_cast<int64_t>(pair) * nchunk * (PW * PW) + threadIdx.x;
    double h = 0;
    for (int c = 0; c < nchunk; ++c) h += Hp[static_cast<int64_t>(c) * PW * PW];
    double w = (i == j) ? 1.0 : 0.0;
    Hs[0][i][j] = h;
    Ws[0][i][j] = w;
    if (threadIdx.x == 0) s_need = 0;
    __syncthreads();
    if (i < j) {
        const double hii = Hs[0][i][i], hjj = Hs[0][j][j];
        if (hii > 0 && hjj > 0 && fabs(h) > tol * sqrt(hii) * sqrt(hjj)) s_need = 1;
    }
    __syncthreads();
    if (!s_need) {
        if (threadIdx.x == 0) flag[pair] = 0;
        return;
    }
    int cur = 0;
    for (int sw = 0; sw < inner_sweeps; ++sw) {
        for (int step = 0; step < PW - 1; ++step) {
            int ip, jp;
            bool il, jl;
            inner_partner(step, i, ip, il);
            inner_partner(step, j, jp, jl);
            double ci, si, cj, sj;
            {
                const int a = il ? i : ip, b = il ? ip : i;
                fast_rotation(Hs[cur][a][a], Hs[cur][b][b], Hs[cur][a][b], ci, si);
                if (il) si = -si;   // lower index: new = c * own - s * partner
            }
            {
                const int a = jl ? j : jp, b = jl ? jp : j;
                fast_rotation(Hs[cur][a][a], Hs[cur][b][b], Hs[cur][a][b], cj, sj);
                if (jl) sj = -sj;
            }
            const double h_ij = h;
            const double h_ijp = Hs[cur][i][jp];
            const double h_ipj = Hs[cur][ip][j];
            const double h_ipjp = Hs[cur][ip][jp];
            const double w_ijp = Ws[cur][i][jp];
            h = ci * (cj * h_ij + sj * h_ijp) + si * (cj * h_ipj + sj * h_ipjp);
            w = cj * w + sj * w_ijp;
            const int nxt = cur ^ 1;
            Hs[nxt][i][j] = h;
            Ws[nxt][i][j] = w;
            __syncthreads();
            cur = nxt;
        }
    }
    Wout[static_cast<int64_t>(pair) * PW * PW + threadIdx.x] = w;
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
            int* sweeps_out, int* host_counter, hipStream_t st, hipStream_t copy_st) {
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
            hipLaunchKernelGGL(k_eig_gram, dim3(npairs, nchunk), dim3(256), 0, st, X, ld, pr, nblk, Hpart,
                               nchunk);
            hipLaunchKernelGGL(k_eig_solve, dim3(npairs), dim3(PW * PW), 0, st, Hpart, nchunk, pr, nblk, W,
                               flag, rot + sweep, tol, inner_sweeps);
            hipLaunchKernelGGL(k_eig_update, dim3(npairs, nupd), dim3(UPD_ROWS), 0, st, X, ld, pr, nblk,
                               W, flag);
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
