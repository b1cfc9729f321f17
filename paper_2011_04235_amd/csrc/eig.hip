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
// A pair whose columns are already orthogonal to `tol` (cosine) is left alone; a problem is
// done after a sweep with no rotated pair. Before every sweep the columns of X are reordered
// by descending norm (de Rijk's ordering), which saves sweeps; X X^T, and so the result, does
// not depend on the order.
//
// Several independent problems ("jobs") advance together. By default a round is two launches:
// the column update of the previous round fused with this round's partial Grams
// (k_eig_round, on two iterates that alternate by round), then the pair solves; the
// three-launch form (partial Grams, pair solves, column updates on one iterate) gives the
// same results bitwise. Each launch's workgroups are spread over the jobs still inside their
// sweep, found from prefix sums of the per-job workgroup counts. Jobs
// with fewer blocks have fewer rounds per sweep and sit out the remaining rounds. A done job
// returns at once from every kernel, so a fixed launch sequence per sweep serves any mix of
// converged and running jobs (and can be replayed from a captured graph).
#include <algorithm>
#include <cfloat>

#include "device_common.h"
#include "kernels.h"

namespace fastpi {

constexpr int BW = 16;
constexpr int PW = 2 * BW;         // columns in a pair
constexpr int UPD_ROWS = 128;      // rows per update workgroup
constexpr int ST_ROT = kEigStRot, ST_DONE = kEigStDone, ST_SWEEPS = kEigStSweeps, ST_CAPPED = kEigStCapped,
              ST_TOTAL = kEigStTotal, ST_WORDS = kEigStateWords;

// largest j < nact with pre[j] <= bid (the job owning flattened workgroup bid)
__device__ __forceinline__ int job_of(const int* __restrict__ pre, int nact, int bid) {
    int lo = 0, hi = nact - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= bid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_eig_init(const EigJob* __restrict__ jobs) {
    const EigJob& J = jobs[blockIdx.y];
    const int64_t n = J.ld * J.ld;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int64_t r = e % J.ld, c = e / J.ld;
        J.X[e] = (r < J.q && c < J.q) ? J.G[r * J.q + c] : 0.0;
    }
}

// Column norms of X: the eigenvalue estimates at the end, and the keys of the column order
// before every sweep (then with the state: finished jobs are skipped). Non-finite values
// sort last so the order stays a permutation.
__global__ void k_eig_norms(const EigJob* __restrict__ jobs, const int* __restrict__ state) {
    if (state && state[ST_WORDS * blockIdx.y + ST_DONE]) return;
    const EigJob& J = jobs[blockIdx.y];
    const int lane = threadIdx.x % kWave;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (c >= J.ld) return;
    double acc = 0;
    for (int64_t r = lane; r < J.q; r += kWave) {
        const double v = J.X[c * J.ld + r];
        acc += v * v;
    }
    acc = wave_sum(acc);
    if (lane == 0) J.lam[c] = (c < J.q && isfinite(acc)) ? (J.squared ? acc : sqrt(acc)) : -DBL_MAX;
}

// lam[ld] = (ld eps)^2 ld max_c ||x_c||^2 over the starting columns: columns of X whose
// squared norm is below it are rounding noise of a (numerically) zero eigenvalue and are
// treated as converged (their cosines with anything are meaningless). For X = G V,
// ||x_c|| = lambda_c, whose rounding level is ~ ld eps lambda_1 with lambda_1 <=
// sqrt(ld) max_c ||G_c||; for X = R^T the columns are at most as large.
__global__ __launch_bounds__(256) void k_eig_floor(const EigJob* __restrict__ jobs) {
    const EigJob& J = jobs[blockIdx.x];
    __shared__ double red[256];
    double mx = 0;
    for (int64_t c = threadIdx.x; c < J.ld; c += blockDim.x) mx = J.lam[c] > mx ? J.lam[c] : mx;
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w && red[threadIdx.x + w] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double e = static_cast<double>(J.ld) * DBL_EPSILON;
        const double mx2 = J.squared ? red[0] : red[0] * red[0];   // largest squared column norm
        J.lam[J.ld] = isfinite(red[0]) ? e * e * static_cast<double>(J.ld) * mx2 : 0.0;
    }
}

// Column order of the next sweep: the columns by descending norm (J.lam, from k_eig_norms;
// ties by index, so the order is deterministic), one workgroup per job, bitonic sort in LDS:
// FP64 keys up to order kSortExact, FP32 keys (the order of norms equal to FP32 rounding
// falls back to the index) up to kSortMax. The key type depends on the job's own order
// only, so a matrix is ordered alike alone and in a batch. Jobs above kSortMax columns (no
// reordering scratch) keep their order.
constexpr int kSortExact = 4096;
constexpr int kSortMax = 16384;
template <typename K>
__device__ void bitonic_desc(K* key, int* idx, int n) {
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < n / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const K klo = key[lo], khi = key[hi];
                const int ilo = idx[lo], ihi = idx[hi];
                // (key descending, index ascending): hi goes before lo
                const bool hi_first = khi > klo || (khi == klo && ihi < ilo);
                if (hi_first == up) {
                    key[lo] = khi;
                    key[hi] = klo;
                    idx[lo] = ihi;
                    idx[hi] = ilo;
                }
            }
            __syncthreads();
        }
    }
}
__global__ __launch_bounds__(1024) void k_eig_sort_cols(const EigJob* __restrict__ jobs,
                                                        const int* __restrict__ state) {
    constexpr int EXACT_BYTES = kSortExact * (sizeof(double) + sizeof(int));
    constexpr int WIDE_BYTES = kSortMax * (sizeof(float) + sizeof(int));
    __shared__ __align__(16) unsigned char sm[EXACT_BYTES > WIDE_BYTES ? EXACT_BYTES : WIDE_BYTES];
    const int j = blockIdx.x;
    if (state[ST_WORDS * j + ST_DONE]) return;
    const EigJob& J = jobs[j];
    const int ld = static_cast<int>(J.ld);
    if (!J.Xs) return;
    int n = 1;
    while (n < ld) n <<= 1;
    int* idx;
    if (ld <= kSortExact) {
        double* key = reinterpret_cast<double*>(sm);
        idx = reinterpret_cast<int*>(sm + kSortExact * sizeof(double));
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            key[i] = i < ld ? J.lam[i] : -DBL_MAX;
            idx[i] = i;
        }
        __syncthreads();
        bitonic_desc(key, idx, n);
    } else {
        float* key = reinterpret_cast<float*>(sm);
        idx = reinterpret_cast<int*>(sm + kSortMax * sizeof(float));
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            // FP32 of the norm, saturated (a norm above FLT_MAX keeps its place among the largest)
            key[i] = i < ld ? static_cast<float>(fmax(fmin(J.lam[i], static_cast<double>(FLT_MAX)), -static_cast<double>(FLT_MAX)))
                            : -FLT_MAX;
            idx[i] = i;
        }
        __syncthreads();
        bitonic_desc(key, idx, n);
    }
    for (int i = threadIdx.x; i < ld; i += blockDim.x) J.perm[i] = idx[i];
}

// Xs[:, i] = X[:, perm[i]] (one wave per column), then (second launch) X = Xs.
__global__ __launch_bounds__(256) void k_eig_gather_cols(const EigJob* __restrict__ jobs,
                                                         const int* __restrict__ state) {
    const int j = blockIdx.y;
    if (state[ST_WORDS * j + ST_DONE]) return;
    const EigJob& J = jobs[j];
    if (!J.Xs) return;
    const int64_t ld = J.ld;
    const int lane = threadIdx.x % kWave;
    for (int64_t c = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave; c < ld;
         c += static_cast<int64_t>(gridDim.x) * (blockDim.x / kWave)) {
        const double* src = J.X + static_cast<int64_t>(J.perm[c]) * ld;
        double* dst = J.Xs + c * ld;
        for (int64_t r = lane; r < ld; r += kWave) dst[r] = src[r];
    }
}
__global__ __launch_bounds__(256) void k_eig_copy_back(const EigJob* __restrict__ jobs,
                                                       const int* __restrict__ state) {
    const int j = blockIdx.y;
    if (state[ST_WORDS * j + ST_DONE]) return;
    const EigJob& J = jobs[j];
    if (!J.Xs) return;
    const int64_t n = J.ld * J.ld;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        J.X[e] = J.Xs[e];
}

// Partial Gram of one pair over one row chunk of X. Wave w accumulates the 32 x 32 product
// over a quarter of the chunk's rows in 4 x 4 register blocks (lane -> block); the four wave
// partials are then summed in wave order.
template <int ROWS>
__global__ __launch_bounds__(256) void k_eig_gram(const EigJob* __restrict__ jobs,
                                                  const int* __restrict__ pre, int nact,
                                                  const int* __restrict__ state, int round) {
    constexpr int YS = ROWS * (PW + 1);
    constexpr int RS = 4 * PW * PW;
    __shared__ double smem[YS > RS ? YS : RS];
    double (*Y)[PW + 1] = reinterpret_cast<double (*)[PW + 1]>(smem);
    const int j = job_of(pre, nact, blockIdx.x);
    if (state[ST_WORDS * j + ST_DONE]) return;
    const EigJob& J = jobs[j];
    const int local = blockIdx.x - pre[j];
    const int pair = local / J.nchunk, ch = local % J.nchunk;
    int bi, bj;
    round_robin_pair(round, pair, J.nbe, bi, bj);
    const bool hasJ = bj < J.nblk;   // the odd block out is paired with 16 zero columns
    const int64_t ld = J.ld;
    const int64_t r0 = static_cast<int64_t>(ch) * ROWS;
    const int nr = static_cast<int>(min<int64_t>(ROWS, ld - r0));
    const double* X = J.X;
    // all loads of the tile in flight at once, then the LDS stores
    constexpr int PER = ROWS * PW / 256;
    double v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        const int c = e / ROWS, r = e % ROWS;
        const int col = c < BW ? bi * BW + c : bj * BW + (c - BW);
        v[k] = (r < nr && (c < BW || hasJ)) ? X[static_cast<int64_t>(col) * ld + r0 + r] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        Y[e % ROWS][e / ROWS] = v[k];
    }
    __syncthreads();
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int ra = (lane / 8) * 4, cb = (lane % 8) * 4;
    double acc[4][4] = {};
    constexpr int QR = ROWS / 4;
    for (int r = wave * QR; r < wave * QR + QR; ++r) {
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            x[u] = Y[r][ra + u];
            y[u] = Y[r][cb + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int w = 0; w < 4; ++w) acc[u][w] += x[u] * y[w];
    }
    __syncthreads();   // Y is reused for the wave partials
    double* part = smem + wave * PW * PW;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) part[(ra + u) * PW + cb + w] = acc[u][w];
    __syncthreads();
    double* Hp = J.Hpart + (static_cast<int64_t>(pair) * J.nchunk + ch) * (PW * PW);
#pragma unroll
    for (int k = 0; k < PW * PW / 256; ++k) {
        const int e = threadIdx.x + k * 256;
        Hp[e] = ((smem[e] + smem[PW * PW + e]) + smem[2 * PW * PW + e]) + smem[3 * PW * PW + e];
    }
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
__device__ __forceinline__ void rutishauser_rotation(double hpp, double hqq, double hpq, double& c, double& s) {
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
// The same (smaller) rotation from the double angle, with a shorter dependency chain: for
// d = hqq - hpp and r = sqrt(d^2 + 4 hpq^2), cos 2theta = |d| / r in [0, 1], so
// c^2 = (1 + cos 2theta) / 2 and s = sign(d) hpq / (r c) (sign(0) = +1), c^2 + s^2 = 1.
// The identity (c, s) = (1, 0) unless `live` and the coupling exceeds rounding level.
// Straight-line code with selects; where d^2 + 4 hpq^2 leaves the normal range the tangent
// form is taken instead (rare: one branch at the end).
__device__ __forceinline__ void fast_rotation(double hpp, double hqq, double hpq, bool live, double& c, double& s) {
    const double ahpq = fabs(hpq);
    const bool rot = live && hpq != 0.0 && ahpq * ahpq > 0.25 * DBL_EPSILON * DBL_EPSILON * fabs(hpp) * fabs(hqq);
    const double d = hqq - hpp;
    const double r2 = fma(d, d, 4.0 * hpq * hpq);
    const bool normal = r2 > 1e-290 && r2 < 1e290;
    const double rr = rsq3(normal ? r2 : 1.0);      // 1 / r
    const double h = fma(0.5 * fabs(d), rr, 0.5);  // c^2
    const double rc = rsq3(h);                     // 1 / c
    c = rot ? h * rc : 1.0;
    s = rot ? (d < 0 ? -hpq : hpq) * (rr * rc) : 0.0;
    if (rot && !normal) rutishauser_rotation(hpp, hqq, hpq, c, s);
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

// LDS slot of H[i][j] (and W[i][j]) in the pair solve: rows LS = 40 doubles apart, the even
// columns of a row in its first 16 doubles and the odd ones in the next 16 (column 2k + 1 at
// 16 + (k + 15) mod 16). The 16 lanes of a quarter wave share a row pair and, in a step, write
// the next slots of the even (or odd) columns, read their own adjacent columns and read the
// diagonal blocks of 16 distinct rows: with this map each of these accesses touches 16
// distinct 8-byte bank pairs (and rows two apart land 16 pairs apart), where a plain
// row-major layout serialises them two to four ways.
constexpr int LS = 40;
__device__ __forceinline__ int slot(int i, int j) { return i * LS + ((j & 1) ? 16 + (((j >> 1) + 15) & 15) : (j >> 1)); }

// One workgroup of 256 threads per pair. Thread (a, b) keeps the 2x2 blocks
// H[2a:2a+2][2b:2b+2] and W[2a:2a+2][2b:2b+2] in registers (H indexed by slots on both
// sides, W by input column and slot), with a copy of H in LDS. In a step every thread
// computes the rotation of its column slot pair b from the diagonal block in LDS and takes
// that of its row slot pair a from lane a of its wave by a shuffle (so all threads use
// bitwise the same rotations), applies J_a^T (.) J_b to its H block and (.) J_b to its W
// block in registers, and scatters the blocks to their next slots through the other LDS
// buffer: one barrier per step. Runs in the calling workgroup: job j's pair `pair` from its
// partial Grams at J.Hpart, the rotations to Wg and the rotated flag to *flagp; lds holds
// 4 * PW * LS doubles.
constexpr int kSolveLds = 4 * PW * LS;
__device__ __forceinline__ void pair_solve(const EigJob& J, int j, int pair, double* __restrict__ Wg,
                                           int* __restrict__ flagp, int* __restrict__ state, int inner_sweeps,
                                           double* lds, int& s_need) {
    double (*Hs)[PW * LS] = reinterpret_cast<double (*)[PW * LS]>(lds);
    double (*Ws)[PW * LS] = reinterpret_cast<double (*)[PW * LS]>(lds + 2 * PW * LS);
    const int nchunk = J.nchunk;
    const double tol = J.tol;
    const double* Hp = J.Hpart + static_cast<int64_t>(pair) * nchunk * (PW * PW);
    {
        // H = sum of the partial Grams in chunk order, up to 12 chunks' loads in flight at once
        constexpr int CG = 12;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int c0 = 0; c0 < nchunk; c0 += CG) {
            double v[CG][4];
#pragma unroll
            for (int u = 0; u < CG; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    v[u][k] = c0 + u < nchunk ? Hp[static_cast<int64_t>(c0 + u) * PW * PW + threadIdx.x + k * 256] : 0.0;
#pragma unroll
            for (int u = 0; u < CG; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (c0 + u < nchunk) acc[k] += v[u][k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = threadIdx.x + k * 256;
            Hs[0][slot(e / PW, e % PW)] = acc[k];
        }
    }
    if (threadIdx.x == 0) s_need = 0;
    __syncthreads();
    const double nf = J.lam[J.ld];
    {
        int need = 0;
        for (int e = threadIdx.x; e < PW * PW; e += 256) {
            const int i = e / PW, k = e % PW;
            if (i < k) {
                const double hii = Hs[0][slot(i, i)], hkk = Hs[0][slot(k, k)], hik = Hs[0][slot(i, k)];
                if (hii > nf && hkk > nf && hik * hik > tol * tol * (hii * hkk)) need = 1;
            }
        }
        if (need) s_need = 1;
    }
    __syncthreads();
    if (!s_need) {
        if (threadIdx.x == 0) *flagp = 0;
        return;
    }
    const int a = threadIdx.x / (PW / 2), b = threadIdx.x % (PW / 2);
    const int r0 = 2 * a, r1 = 2 * a + 1, c0 = 2 * b, c1 = 2 * b + 1;
    double h00 = Hs[0][slot(r0, c0)], h01 = Hs[0][slot(r0, c1)], h10 = Hs[0][slot(r1, c0)], h11 = Hs[0][slot(r1, c1)];
    double w00 = (r0 == c0), w01 = (r0 == c1), w10 = (r1 == c0), w11 = (r1 == c1);
    // slot permutation of the four rows/columns this thread owns
    const int pr0 = inner_next_slot(r0), pr1 = inner_next_slot(r1);
    const int pc0 = inner_next_slot(c0), pc1 = inner_next_slot(c1);
    int cur = 0;
    for (int sw = 0; sw < inner_sweeps; ++sw) {
        for (int step = 0; step < PW - 1; ++step) {
            // the rotations of this thread's column pair b (computed here from its diagonal
            // 2 x 2 block) and row pair a (computed by lane a of the same wave, whose column
            // pair is a: every wave holds all 16 rotations, so all threads apply bitwise the
            // same ones)
            double cb, sb;
            {
                const double bpp = Hs[cur][slot(c0, c0)], bpq = Hs[cur][slot(c0, c1)], bqq = Hs[cur][slot(c1, c1)];
                fast_rotation(bpp, bqq, bpq, bpp > nf && bqq > nf, cb, sb);
            }
            const double ca = __shfl(cb, a, kWave), sa = __shfl(sb, a, kWave);
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
            // move to the next step's slots (W rows are input columns and stay); the buffer
            // written here was last read before the previous barrier
            const int nxt = cur ^ 1;
            Hs[nxt][slot(pr0, pc0)] = h00;
            Hs[nxt][slot(pr0, pc1)] = h01;
            Hs[nxt][slot(pr1, pc0)] = h10;
            Hs[nxt][slot(pr1, pc1)] = h11;
            Ws[nxt][slot(r0, pc0)] = w00;
            Ws[nxt][slot(r0, pc1)] = w01;
            Ws[nxt][slot(r1, pc0)] = w10;
            Ws[nxt][slot(r1, pc1)] = w11;
            __syncthreads();
            h00 = Hs[nxt][slot(r0, c0)];
            h01 = Hs[nxt][slot(r0, c1)];
            h10 = Hs[nxt][slot(r1, c0)];
            h11 = Hs[nxt][slot(r1, c1)];
            w00 = Ws[nxt][slot(r0, c0)];
            w01 = Ws[nxt][slot(r0, c1)];
            w10 = Ws[nxt][slot(r1, c0)];
            w11 = Ws[nxt][slot(r1, c1)];
            cur = nxt;
        }
    }
    // after whole sweeps every slot holds its own column again
    Wg[r0 * PW + c0] = w00;
    Wg[r0 * PW + c1] = w01;
    Wg[r1 * PW + c0] = w10;
    Wg[r1 * PW + c1] = w11;
    if (threadIdx.x == 0) {
        *flagp = 1;
        atomicAdd(state + ST_WORDS * j + ST_ROT, 1);
    }
}

// par: the parity slot of the rotations and flags (the round's parity in the two-launch
// rounds, 0 in the three-launch rounds)
__global__ __launch_bounds__(256) void k_eig_solve(const EigJob* __restrict__ jobs,
                                                   const int* __restrict__ pre, int nact,
                                                   int* __restrict__ state, int inner_sweeps, int par) {
    __shared__ double lds[kSolveLds];
    __shared__ int s_need;
    const int j = job_of(pre, nact, blockIdx.x);
    if (state[ST_WORDS * j + ST_DONE]) return;
    const EigJob& J = jobs[j];
    const int pair = blockIdx.x - pre[j];
    const int64_t slot = static_cast<int64_t>(par) * J.npairs + pair;
    pair_solve(J, j, pair, J.W + slot * (PW * PW), J.flag + slot, state, inner_sweeps, lds, s_need);
}

// X[:, I u J] <- X[:, I u J] W over a tile of UPD_ROWS rows: the tile and W staged in LDS,
// each thread a 4 x 4 block of the product (rows lane-strided, so stores are coalesced).
__global__ __launch_bounds__(256) void k_eig_update(const EigJob* __restrict__ jobs,
                                                    const int* __restrict__ pre, int nact,
                                                    const int* __restrict__ state, int round) {
    __shared__ double Ws[PW][PW + 1];
    __shared__ double Xs[PW][UPD_ROWS + 1];
    const int j = job_of(pre, nact, blockIdx.x);
    if (state[ST_WORDS * j + ST_DONE]) return;
    const EigJob& J = jobs[j];
    const int local = blockIdx.x - pre[j];
    const int pair = local / J.nupd, rb = local % J.nupd;
    if (J.flag[pair] == 0) return;
    int bi, bj;
    round_robin_pair(round, pair, J.nbe, bi, bj);
    const bool hasJ = bj < J.nblk;
    const int64_t ld = J.ld;
    const int64_t r0 = static_cast<int64_t>(rb) * UPD_ROWS;
    const int nr = static_cast<int>(min<int64_t>(UPD_ROWS, ld - r0));
    double* X = J.X;
    const double* Wg = J.W + static_cast<int64_t>(pair) * PW * PW;
    {
        constexpr int PX = PW * UPD_ROWS / 256, PWW = PW * PW / 256;
        double xv[PX], wv[PWW];
#pragma unroll
        for (int k = 0; k < PWW; ++k) wv[k] = Wg[threadIdx.x + k * 256];
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            const int e = threadIdx.x + k * 256;
            const int c = e / UPD_ROWS, r = e % UPD_ROWS;
            const int col = c < BW ? bi * BW + c : bj * BW + (c - BW);
            xv[k] = (r < nr && (c < BW || hasJ)) ? X[static_cast<int64_t>(col) * ld + r0 + r] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < PWW; ++k) {
            const int e = threadIdx.x + k * 256;
            Ws[e / PW][e % PW] = wv[k];
        }
#pragma unroll
        for (int k = 0; k < PX; ++k) {
            const int e = threadIdx.x + k * 256;
            Xs[e / UPD_ROWS][e % UPD_ROWS] = xv[k];
        }
    }
    __syncthreads();
    constexpr int RL = UPD_ROWS / 4;              // row lanes; rows rl, rl + RL, ...
    const int rl = threadIdx.x % RL, c0 = (threadIdx.x / RL) * 4;
    double acc[4][4] = {};
#pragma unroll 8
    for (int k = 0; k < PW; ++k) {
        double x[4], w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            x[u] = Xs[k][rl + u * RL];
            w[u] = Ws[k][c0 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += x[u] * w[v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int c = c0 + v;
        if (!(c < BW || hasJ)) continue;
        const int col = c < BW ? bi * BW + c : bj * BW + (c - BW);
        double* Xc = X + static_cast<int64_t>(col) * ld + r0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = rl + u * RL;
            if (r < nr) Xc[r] = acc[u][v];
        }
    }
}

// Column update of round t and partial Grams of round t + 1 in one launch, on two iterates
// (X and Xs) that alternate by round; the pair solves of round t + 1 follow in k_eig_solve.
// The workgroups are laid out by the pairs of round t + 1 and the row chunks, as the partial
// Grams. Workgroup (pair (a, b), chunk) computes the chunk's rows of blocks a and b after
// round t's rotations, each from the pair of round t that held it (read from one iterate,
// written to the other, so no workgroup reads what another one writes), keeps them in LDS and
// writes the pair's partial Gram of round t + 1 over them. t = -1 is the first launch of a
// sweep (the blocks as reordered into Xs, no update); in a job's last round (t + 1 = its
// rounds per sweep) only the update runs, laid out by the pairs of round 0. A sweep has an
// odd number of rounds, so it starts from X, reorders into Xs and ends in X again. Rotations
// and rotated flags alternate by round parity as well (round t's are read while round t + 1's
// are written).
template <int ROWS>
__global__ __launch_bounds__(256) void k_eig_round(const EigJob* __restrict__ jobs,
                                                   const int* __restrict__ pre, int nact,
                                                   const int* __restrict__ state, int t) {
    constexpr int YS = ROWS * (PW + 1);   // the two blocks' new rows
    constexpr int WS = 2 * PW * PW;       // round t's rotations of the pairs that held them
    constexpr int A1 = YS + WS, A2 = 4 * PW * PW;
    __shared__ double smem[A1 > A2 ? A1 : A2];
    __shared__ int s_flag[2];
    double (*Y)[PW + 1] = reinterpret_cast<double (*)[PW + 1]>(smem);
    const int j = job_of(pre, nact, blockIdx.x);
    if (state[ST_WORDS * j + ST_DONE]) return;
    const EigJob& J = jobs[j];
    const int rounds = J.nbe - 1;
    const int local = blockIdx.x - pre[j];
    const int pair = local / J.nchunk, ch = local % J.nchunk;
    int ba, bb;
    round_robin_pair((t + 1) % rounds, pair, J.nbe, ba, bb);
    const int64_t ld = J.ld;
    const int64_t r0 = static_cast<int64_t>(ch) * ROWS;
    const int nr = static_cast<int>(min<int64_t>(ROWS, ld - r0));
    const int tid = threadIdx.x;
    if (t < 0) {
        const bool hasB = bb < J.nblk;   // the odd block out is paired with 16 zero columns
        constexpr int PER = ROWS * PW / 256;
        double v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + k * 256;
            const int c = e / ROWS, r = e % ROWS;
            const int col = c < BW ? ba * BW + c : bb * BW + (c - BW);
            v[k] = (r < nr && (c < BW || hasB)) ? J.Xs[static_cast<int64_t>(col) * ld + r0 + r] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + k * 256;
            Y[e % ROWS][e / ROWS] = v[k];
        }
    } else {
        const double* Xin = (t & 1) ? J.X : J.Xs;
        double* Xout = (t & 1) ? J.Xs : J.X;
        const int64_t par = t & 1;
        const double* Wt = J.W + par * J.npairs * (PW * PW);
        const int* ft = J.flag + par * J.npairs;
        double* Wl = smem + YS;
        int pr[2], lo[2], hi[2], off[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int x = h ? bb : ba;
            int other;
            round_robin_find(t, x, J.nbe, pr[h], other);
            lo[h] = min(x, other);
            hi[h] = max(x, other);
            off[h] = x < other ? 0 : BW;
        }
        {
            // both pairs' rotations (stale where a pair did not rotate: then unused)
            constexpr int PWW = WS / 256;
            double wv[PWW];
#pragma unroll
            for (int k = 0; k < PWW; ++k) {
                const int e = tid + k * 256;
                wv[k] = Wt[static_cast<int64_t>(pr[e / (PW * PW)]) * (PW * PW) + e % (PW * PW)];
            }
#pragma unroll
            for (int k = 0; k < PWW; ++k) Wl[tid + k * 256] = wv[k];
            if (tid < 2) s_flag[tid] = ft[pr[tid]];
        }
        __syncthreads();
        // item (block h, row r): one thread per row of each block; a wave's items share h
        for (int e = tid; e < 2 * ROWS; e += 256) {
            const int h = e / ROWS, r = e % ROWS;
            const int x = h ? bb : ba;
            const bool live = x < J.nblk && r < nr;
            double out[BW];
            if (!s_flag[h]) {
                // the pair left alone in round t: the block is unchanged
#pragma unroll
                for (int c = 0; c < BW; ++c)
                    out[c] = live ? Xin[static_cast<int64_t>(x * BW + c) * ld + r0 + r] : 0.0;
            } else {
                double xin[PW];
#pragma unroll
                for (int c = 0; c < PW; ++c) {
                    const int blk = c < BW ? lo[h] : hi[h];
                    xin[c] = (live && blk < J.nblk) ? Xin[static_cast<int64_t>(blk * BW + c % BW) * ld + r0 + r] : 0.0;
                }
                const double* Wh = Wl + h * (PW * PW) + off[h];
#pragma unroll
                for (int c = 0; c < BW; ++c) out[c] = 0.0;
#pragma unroll
                for (int k = 0; k < PW; ++k)
#pragma unroll
                    for (int c = 0; c < BW; ++c) out[c] += xin[k] * Wh[k * PW + c];
            }
            if (live) {
#pragma unroll
                for (int c = 0; c < BW; ++c) Xout[static_cast<int64_t>(x * BW + c) * ld + r0 + r] = out[c];
            }
#pragma unroll
            for (int c = 0; c < BW; ++c) Y[r][h * BW + c] = out[c];
        }
    }
    if (t + 1 >= rounds) return;   // the job's last round: update only
    __syncthreads();
    // partial Gram of round t + 1's pair over the chunk, as k_eig_gram
    const int lane = tid % kWave, wave = tid / kWave;
    const int ra = (lane / 8) * 4, cb = (lane % 8) * 4;
    double acc[4][4] = {};
    constexpr int QR = ROWS / 4;
    for (int r = wave * QR; r < wave * QR + QR; ++r) {
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            x[u] = Y[r][ra + u];
            y[u] = Y[r][cb + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int w = 0; w < 4; ++w) acc[u][w] += x[u] * y[w];
    }
    __syncthreads();
    double* part = smem + wave * PW * PW;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) part[(ra + u) * PW + cb + w] = acc[u][w];
    __syncthreads();
    double* Hp = J.Hpart + (static_cast<int64_t>(pair) * J.nchunk + ch) * (PW * PW);
#pragma unroll
    for (int k = 0; k < PW * PW / 256; ++k) {
        const int e = tid + k * 256;
        Hp[e] = ((smem[e] + smem[PW * PW + e]) + smem[2 * PW * PW + e]) + smem[3 * PW * PW + e];
    }
}

// End of a sweep: a job whose sweep rotated nothing is done; one that reached the sweep cap
// is done and flagged. The last word says whether every job is done.
__global__ __launch_bounds__(256) void k_eig_sweep_end(const EigJob* __restrict__ jobs, int njobs,
                                                       int* __restrict__ state, int max_sweeps) {
    __shared__ int s_all;
    if (threadIdx.x == 0) s_all = 1;
    __syncthreads();
    for (int j = threadIdx.x; j < njobs; j += blockDim.x) {
        int* sj = state + ST_WORDS * j;
        if (!sj[ST_DONE]) {
            sj[ST_SWEEPS] += 1;
            sj[ST_TOTAL] += sj[ST_ROT];
            if (sj[ST_ROT] == 0) {
                sj[ST_DONE] = 1;
            } else if (sj[ST_SWEEPS] >= max_sweeps) {
                sj[ST_DONE] = 1;
                sj[ST_CAPPED] = 1;
                if (jobs[j].status) atomicOr(jobs[j].status, 2);
            }
            sj[ST_ROT] = 0;
        }
        if (!sj[ST_DONE]) s_all = 0;   // every writer stores 0
    }
    __syncthreads();
    if (threadIdx.x == 0) state[ST_WORDS * njobs] = s_all;
}

// order of the t largest eigenvalues (descending, ties to the lower column)
__global__ __launch_bounds__(1024) void k_eig_select(const EigJob* __restrict__ jobs) {
    const EigJob& J = jobs[blockIdx.x];
    const double* lam = J.lam;
    for (int64_t c = threadIdx.x; c < J.q; c += blockDim.x) {
        const double lc = lam[c];
        int64_t rk = 0;
        for (int64_t d = 0; d < J.q; ++d) {
            const double ld_ = lam[d];
            rk += (ld_ > lc) || (ld_ == lc && d < c);
        }
        if (rk < J.t) J.order[rk] = static_cast<int>(c);
    }
}

// vecs (q x t, row-major): the normalised columns of X; vals (t): their norms
__global__ void k_eig_output(const EigJob* __restrict__ jobs) {
    const EigJob& J = jobs[blockIdx.y];
    const int64_t n = J.q * J.t;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int64_t r = e / J.t, k = e % J.t;
        const int oc = J.order[k];
        const double l = J.lam[oc];
        const double inv = l > 0 ? (J.squared ? 1.0 / sqrt(l) : 1.0 / l) : 0.0;
        J.vecs[e] = J.X[static_cast<int64_t>(oc) * J.ld + r] * inv;
        if (r == 0) J.vals[k] = l > 0 ? l : 0.0;
    }
}

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------
int64_t eig_padded_order(int64_t q) { return ((q + BW - 1) / BW) * BW; }

int eig_gram_rows_valid(int rows) { return rows == 64 || rows == 128 || rows == 256; }

static void job_shape(int64_t q, int gram_rows, int64_t& ld, int& nblk, int& nbe, int& npairs,
                      int& nchunk, int& nupd) {
    ld = eig_padded_order(q);
    nblk = static_cast<int>(ld / BW);
    nbe = nblk + (nblk & 1);   // even number of slots (the extra one is a dummy)
    npairs = nbe / 2;
    nchunk = static_cast<int>((ld + gram_rows - 1) / gram_rows);
    nupd = static_cast<int>((ld + UPD_ROWS - 1) / UPD_ROWS);
}

size_t eig_job_doubles(int64_t q, int gram_rows) {
    int64_t ld;
    int nblk, nbe, npairs, nchunk, nupd;
    job_shape(q, gram_rows, ld, nblk, nbe, npairs, nchunk, nupd);
    return static_cast<size_t>(ld * ld + static_cast<int64_t>(npairs) * nchunk * PW * PW +
                               2 * static_cast<int64_t>(npairs) * PW * PW + ld + 32 + (ld <= kSortMax ? ld * ld : 0));
}

size_t eig_job_ints(int64_t q) {
    const int64_t ld = eig_padded_order(q);
    const int64_t npairs = (ld / BW + 1) / 2;
    return static_cast<size_t>(2 * npairs + 2 * ld + 32);
}

EigJob eig_make_job(const double* G, double* A, int64_t q, int64_t t, double* vals, double* vecs,
                    double* ws, int* iws, int* status, double tol, int gram_rows, int tag) {
    EigJob J{};
    job_shape(q, gram_rows, J.ld, J.nblk, J.nbe, J.npairs, J.nchunk, J.nupd);
    J.G = G;
    J.A = A;
    J.vals = vals;
    J.vecs = vecs;
    J.q = q;
    J.t = t;
    J.X = ws;
    J.Hpart = J.X + J.ld * J.ld;
    J.W = J.Hpart + static_cast<int64_t>(J.npairs) * J.nchunk * PW * PW;
    J.lam = J.W + 2 * static_cast<int64_t>(J.npairs) * PW * PW;
    J.Xs = J.ld <= kSortMax ? J.lam + J.ld + 32 : nullptr;
    J.flag = iws;
    J.order = iws + 2 * J.npairs;
    J.perm = J.order + J.ld;
    J.status = status;
    J.tol = tol > 0 ? tol : static_cast<double>(J.ld) * DBL_EPSILON;
    J.tag = tag;
    return J;
}

void eig_set_free(EigSet& es) {
    if (es.jobs) hipFree(es.jobs);
    if (es.pre) hipFree(es.pre);
    if (es.state) hipFree(es.state);
    if (es.pstate) hipFree(es.pstate);
    if (es.host_state) hipHostFree(es.host_state);
    es = EigSet{};
}

int eig_set_create(EigSet& es, std::vector<EigJob> jobs, int gram_rows, bool precond, bool fused,
                   hipStream_t st) {
    eig_set_free(es);
    es.gram_rows = gram_rows;
    // the pivoted-Cholesky start per job: the jobs given scratch for it take it
    bool any = false;
    for (EigJob& J : jobs) {
        J.squared = precond && J.A ? 1 : 0;
        any = any || J.squared;
        if (!J.Xs) fused = false;
    }
    es.precond = any ? 1 : 0;
    es.fused = fused ? 1 : 0;
    std::stable_sort(jobs.begin(), jobs.end(),
                     [](const EigJob& x, const EigJob& y) { return x.nbe > y.nbe; });
    const int nj = static_cast<int>(jobs.size());
    es.njobs = nj;
    es.host = jobs;
    if (nj == 0) return FASTPI_OK;
    es.rounds = jobs[0].nbe - 1;
    std::vector<int> pre(3 * (nj + 1), 0);
    for (int j = 0; j < nj; ++j) {
        const EigJob& J = jobs[j];
        pre[j + 1] = pre[j] + J.npairs * J.nchunk;
        pre[(nj + 1) + j + 1] = pre[(nj + 1) + j] + J.npairs;
        pre[2 * (nj + 1) + j + 1] = pre[2 * (nj + 1) + j] + J.npairs * J.nupd;
        es.max_ld = std::max(es.max_ld, J.ld);
        es.max_q = std::max(es.max_q, J.q);
    }
    for (int t = 0; t < es.rounds; ++t) {
        int na = 0;
        while (na < nj && jobs[na].nbe - 1 > t) ++na;
        es.nact.push_back(na);
        es.g_gram.push_back(pre[na]);
        es.g_solve.push_back(pre[(nj + 1) + na]);
        es.g_upd.push_back(pre[2 * (nj + 1) + na]);
    }
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(EigJob) * nj) != hipSuccess) return FASTPI_ENOMEM;
    es.jobs = static_cast<EigJob*>(p);
    if (hipMalloc(&p, sizeof(int) * pre.size()) != hipSuccess) return FASTPI_ENOMEM;
    es.pre = static_cast<int*>(p);
    if (hipMalloc(&p, sizeof(int) * (ST_WORDS * nj + ST_WORDS)) != hipSuccess) return FASTPI_ENOMEM;
    es.state = static_cast<int*>(p);
    if (hipMalloc(&p, sizeof(int) * (2 * nj + 2)) != hipSuccess) return FASTPI_ENOMEM;
    es.pstate = static_cast<int*>(p);
    if (hipHostMalloc(&p, sizeof(int) * (ST_WORDS * nj + ST_WORDS), hipHostMallocDefault) != hipSuccess)
        return FASTPI_ENOMEM;
    es.host_state = static_cast<int*>(p);
    std::fill(es.host_state, es.host_state + ST_WORDS * nj + ST_WORDS, 0);
    if (hipMemcpyAsync(es.jobs, es.host.data(), sizeof(EigJob) * nj, hipMemcpyHostToDevice, st) != hipSuccess)
        return FASTPI_EHIP;
    if (hipMemcpyAsync(es.pre, pre.data(), sizeof(int) * pre.size(), hipMemcpyHostToDevice, st) != hipSuccess)
        return FASTPI_EHIP;
    // the pageable sources above must outlive the copies
    if (hipStreamSynchronize(st) != hipSuccess) return FASTPI_EHIP;
    return FASTPI_OK;
}

void eig_begin(const EigSet& es, hipStream_t st) {
    if (es.njobs == 0) return;
    const unsigned nj = static_cast<unsigned>(es.njobs);
    launch_fill_i32(es.state, ST_WORDS * es.njobs + ST_WORDS, 0, st);
    if (es.precond) {
        pchol_run(es, st);
    } else {
        const unsigned gx = static_cast<unsigned>(std::min<int64_t>((es.max_ld * es.max_ld + 255) / 256, 4096));
        hipLaunchKernelGGL(k_eig_init, dim3(gx, nj), dim3(256), 0, st, es.jobs);
    }
    hipLaunchKernelGGL(k_eig_norms, dim3(static_cast<unsigned>((es.max_ld + 3) / 4), nj), dim3(256), 0, st,
                       es.jobs, nullptr);
    hipLaunchKernelGGL(k_eig_floor, dim3(nj), dim3(256), 0, st, es.jobs);
}

void eig_sweep(const EigSet& es, int max_sweeps, int inner_sweeps, hipStream_t st, KernelTimer* timer) {
    if (es.njobs == 0) return;
    const int nj = es.njobs;
    const int* pg = es.pre;
    const int* ps = es.pre + (nj + 1);
    const int* pu = es.pre + 2 * (nj + 1);
    // the running jobs' column maps by their current norms
    hipLaunchKernelGGL(k_eig_norms, dim3(static_cast<unsigned>((es.max_ld + 3) / 4), nj), dim3(256), 0, st,
                       es.jobs, es.state);
    hipLaunchKernelGGL(k_eig_sort_cols, dim3(nj), dim3(1024), 0, st, es.jobs, es.state);
    const unsigned gc = static_cast<unsigned>(std::min<int64_t>((es.max_ld + 3) / 4, 1024));
    hipLaunchKernelGGL(k_eig_gather_cols, dim3(gc, nj), dim3(256), 0, st, es.jobs, es.state);
    if (es.fused) {
        // the reordered columns stay in Xs: round -1 reads them there
        for (int t = -1; t < es.rounds; ++t) {
            const int tt = t < 0 ? 0 : t;
            const int na = es.nact[tt];
            const dim3 grid(static_cast<unsigned>(es.g_gram[tt]));
            switch (es.gram_rows) {
                case 64:
                    FASTPI_LAUNCH(timer, KT_EIG_ROUND, (k_eig_round<64>), grid, dim3(256), 0, st, es.jobs, pg, na,
                                  es.state, t);
                    break;
                case 256:
                    FASTPI_LAUNCH(timer, KT_EIG_ROUND, (k_eig_round<256>), grid, dim3(256), 0, st, es.jobs, pg, na,
                                  es.state, t);
                    break;
                default:
                    FASTPI_LAUNCH(timer, KT_EIG_ROUND, (k_eig_round<128>), grid, dim3(256), 0, st, es.jobs, pg, na,
                                  es.state, t);
            }
            if (t + 1 < es.rounds)
                FASTPI_LAUNCH(timer, KT_EIG_SOLVE, k_eig_solve, dim3(es.g_solve[t + 1]), dim3(256), 0, st, es.jobs, ps,
                              es.nact[t + 1], es.state, inner_sweeps, (t + 1) & 1);
        }
        hipLaunchKernelGGL(k_eig_sweep_end, dim3(1), dim3(256), 0, st, es.jobs, nj, es.state, max_sweeps);
        return;
    }
    const unsigned gx = static_cast<unsigned>(std::min<int64_t>((es.max_ld * es.max_ld + 255) / 256, 2048));
    hipLaunchKernelGGL(k_eig_copy_back, dim3(gx, nj), dim3(256), 0, st, es.jobs, es.state);
    for (int t = 0; t < es.rounds; ++t) {
        const int na = es.nact[t];
        switch (es.gram_rows) {
            case 64:
                FASTPI_LAUNCH(timer, KT_EIG_GRAM, (k_eig_gram<64>), dim3(es.g_gram[t]), dim3(256), 0, st, es.jobs, pg,
                              na, es.state, t);
                break;
            case 256:
                FASTPI_LAUNCH(timer, KT_EIG_GRAM, (k_eig_gram<256>), dim3(es.g_gram[t]), dim3(256), 0, st, es.jobs, pg,
                              na, es.state, t);
                break;
            default:
                FASTPI_LAUNCH(timer, KT_EIG_GRAM, (k_eig_gram<128>), dim3(es.g_gram[t]), dim3(256), 0, st, es.jobs, pg,
                              na, es.state, t);
        }
        FASTPI_LAUNCH(timer, KT_EIG_SOLVE, k_eig_solve, dim3(es.g_solve[t]), dim3(256), 0, st, es.jobs, ps, na,
                      es.state, inner_sweeps, 0);
        FASTPI_LAUNCH(timer, KT_EIG_UPDATE, k_eig_update, dim3(es.g_upd[t]), dim3(256), 0, st, es.jobs, pu, na,
                      es.state, t);
    }
    hipLaunchKernelGGL(k_eig_sweep_end, dim3(1), dim3(256), 0, st, es.jobs, nj, es.state, max_sweeps);
}

void eig_end(const EigSet& es, hipStream_t st) {
    if (es.njobs == 0) return;
    const unsigned nj = static_cast<unsigned>(es.njobs);
    int64_t max_qt = 0;
    for (const EigJob& J : es.host) max_qt = std::max(max_qt, J.q * J.t);
    hipLaunchKernelGGL(k_eig_norms, dim3(static_cast<unsigned>((es.max_ld + 3) / 4), nj), dim3(256), 0, st,
                       es.jobs, nullptr);
    hipLaunchKernelGGL(k_eig_select, dim3(nj), dim3(1024), 0, st, es.jobs);
    const unsigned gx = static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((max_qt + 255) / 256, 4096)));
    hipLaunchKernelGGL(k_eig_output, dim3(gx, nj), dim3(256), 0, st, es.jobs);
}

int eig_iterate(const EigSet& es, int max_sweeps, int inner_sweeps, hipStream_t st, hipStream_t copy_st,
                KernelTimer* timer, hipGraphExec_t sweep_graph) {
    if (es.njobs == 0) return FASTPI_OK;
    const size_t words = ST_WORDS * es.njobs + ST_WORDS;
    hipEvent_t ev[2];
    if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess) return FASTPI_EHIP;
    if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
        hipEventDestroy(ev[0]);
        return FASTPI_EHIP;
    }
    int rc = FASTPI_OK;
    // reads the state after sweep k (event e) on the side stream
    auto read_state = [&](hipEvent_t e) -> bool {
        if (hipStreamWaitEvent(copy_st, e, 0) != hipSuccess) return false;
        if (hipMemcpyAsync(es.host_state, es.state, sizeof(int) * words, hipMemcpyDeviceToHost, copy_st) !=
            hipSuccess)
            return false;
        return hipStreamSynchronize(copy_st) == hipSuccess;
    };
    bool all_done = false;
    int queued = 0;
    // every job is done after at most max_sweeps sweeps (the cap marks it done)
    for (int sweep = 0; sweep < max_sweeps && !all_done; ++sweep) {
        if (sweep_graph) {
            if (hipGraphLaunch(sweep_graph, st) != hipSuccess) {
                rc = FASTPI_EHIP;
                break;
            }
        } else {
            eig_sweep(es, max_sweeps, inner_sweeps, st, timer);
        }
        if (hipEventRecord(ev[sweep & 1], st) != hipSuccess) {
            rc = FASTPI_EHIP;
            break;
        }
        queued = sweep + 1;
        if (sweep >= 1) {
            // read the previous sweep's state while this one runs
            if (!read_state(ev[(sweep - 1) & 1])) {
                rc = FASTPI_EHIP;
                break;
            }
            all_done = es.host_state[ST_WORDS * es.njobs] != 0;
        }
    }
    // the final state (a sweep queued after convergence changes nothing)
    if (rc == FASTPI_OK && queued > 0 && !read_state(ev[(queued - 1) & 1])) rc = FASTPI_EHIP;
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    return rc;
}

}  // namespace fastpi
