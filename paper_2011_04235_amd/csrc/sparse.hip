// Sparse and block-structured kernels of the incremental updates (Eqs. 2 and 3).
// Every reduction runs in a fixed order (no floating-point atomics), so results are
// reproducible bit for bit.
#include "device_common.h"
#include "kernels.h"

namespace fastpi {

// All sparse products below run over the segments of a compressed structure (see
// Segments): one wave per segment visits its entries in order; owners with one segment are
// written directly, the others through partial rows that k_seg_reduce_* sum in segment
// order. No floating-point atomics, so results are reproducible bit for bit.

// G[a, :] (+)= sum_h S[h, a] S[h, :] for a sparse S given as CSC (segments over its
// columns, rowidx, cval) and CSR (rowptr, colidx, rval): the Gram S^T S, q x q.
constexpr int SG_WAVES = 4;
constexpr int SG_GROUP = 8;   // entries whose first row batches are loaded together
constexpr int SG_LONG = 4;    // row batches of a long row loaded together

// value of lane l (uniform l) for 64-bit integers and doubles
__device__ __forceinline__ int64_t lane_i64(int64_t v, int l) {
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(v), l);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(v >> 32), l);
    return static_cast<int64_t>((static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo));
}
__device__ __forceinline__ double lane_f64(double v, int l) { return __longlong_as_double(lane_i64(__double_as_longlong(v), l)); }

// One wave per (segment, column chunk); the segment's entries are added in order, each entry's
// row in 64-wide batches (lane i takes the row's elements i, i + 64, ...; a row's columns are
// distinct, so the order within an entry does not matter). Memory latency is overlapped without
// changing that order: the entries' rows, values and row extents are read once per 64 entries
// (one per lane), the first batches of SG_GROUP entries are loaded together before they are
// added one entry after the other, and the rest of a long row is loaded SG_LONG batches at a
// time.
__global__ __launch_bounds__(SG_WAVES * 64) void k_sparse_gram(
    SegDev sg, const int* __restrict__ rowidx, const double* __restrict__ cval,
    const int64_t* __restrict__ rowptr, const int* __restrict__ colidx, const double* __restrict__ rval,
    int64_t q, int64_t chunk, double* __restrict__ G, int64_t ldg, int accumulate,
    double* __restrict__ part) {
    extern __shared__ double buf_all[];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t nchunks = (q + chunk - 1) / chunk;
    const int64_t task = static_cast<int64_t>(blockIdx.x) * SG_WAVES + wave;
    if (task >= sg.nseg * nchunks) return;
    const int64_t seg = task / nchunks;
    const int64_t c0 = (task % nchunks) * chunk;
    const int64_t c1 = min(q, c0 + chunk);
    const int64_t a = sg.owner[seg];
    const int pidx = sg.pidx[seg];
    double* buf = buf_all + static_cast<int64_t>(wave) * chunk;
    double* dst = pidx < 0 ? G + a * ldg : part + static_cast<int64_t>(pidx) * q;
    for (int64_t c = c0 + lane; c < c1; c += kWave)
        buf[c - c0] = (pidx < 0 && accumulate) ? dst[c] : 0.0;
    __builtin_amdgcn_wave_barrier();
    const int64_t seg_end = sg.end[seg];
    for (int64_t g0 = sg.begin[seg]; g0 < seg_end; g0 += kWave) {
        const int ne = static_cast<int>(min<int64_t>(kWave, seg_end - g0));
        // every load below reads a valid index (clamped; a segment's matrix has entries, and
        // a row batch's index is clamped into its non-empty row or to entry 0), and the lanes
        // or entries past the end select neutral values: no branches around the loads, so
        // they stay in flight across the adds
        const int64_t h = rowidx[g0 + min(lane, ne - 1)];
        const double va = cval[g0 + min(lane, ne - 1)];
        const int64_t rb = rowptr[h], re = rowptr[h + 1];
        for (int k0 = 0; k0 < ne; k0 += SG_GROUP) {
            // the first row batch of SG_GROUP entries, all loads in flight together
            int fb[SG_GROUP];
            double fv[SG_GROUP];
#pragma unroll
            for (int u = 0; u < SG_GROUP; ++u) {
                const int kc = min(k0 + u, ne - 1);
                const int64_t f = lane_i64(rb, kc) + lane;
                const bool ok = k0 + u < ne && f < lane_i64(re, kc);
                const int64_t fi = ok ? f : 0;
                const int bl = colidx[fi];
                const double vl = rval[fi];
                fb[u] = ok ? bl : -1;
                fv[u] = vl;
            }
#pragma unroll
            for (int u = 0; u < SG_GROUP; ++u) asm volatile("" : "+v"(fb[u]), "+v"(fv[u]));
#pragma unroll
            for (int u = 0; u < SG_GROUP; ++u) {
                const int k = k0 + u;
                if (k >= ne) break;
                const int b = fb[u];
                const double v = fv[u];
                const double ak = lane_f64(va, k);
                if (b >= c0 && b < c1) buf[b - c0] += ak * v;
                const int64_t e = lane_i64(re, k);
                for (int64_t f0 = lane_i64(rb, k) + kWave; f0 < e; f0 += SG_LONG * kWave) {
                    int bq[SG_LONG];
                    double vq[SG_LONG];
#pragma unroll
                    for (int w = 0; w < SG_LONG; ++w) {
                        const int64_t f = f0 + w * kWave + lane;
                        const int64_t fi = f < e ? f : e - 1;
                        const int bl = colidx[fi];
                        const double vl = rval[fi];
                        bq[w] = f < e ? bl : -1;
                        vq[w] = vl;
                    }
                    // all SG_LONG batches arrive before the adds (keeps the compiler from moving
                    // a value's load into the conditional add, behind the earlier adds)
#pragma unroll
                    for (int w = 0; w < SG_LONG; ++w) asm volatile("" : "+v"(bq[w]), "+v"(vq[w]));
#pragma unroll
                    for (int w = 0; w < SG_LONG; ++w)
                        if (bq[w] >= c0 && bq[w] < c1) buf[bq[w] - c0] += ak * vq[w];
                }
                // the next entry may touch the same columns from other lanes
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    }
    for (int64_t c = c0 + lane; c < c1; c += kWave) dst[c] = buf[c - c0];
}

// acc + part[p0 * ld] + part[(p0 + 1) * ld] + ... + part[(p1 - 1) * ld], added in that order
// with eight loads in flight at a time (an owner may have hundreds of segments)
__device__ __forceinline__ double sum_parts_in_order(double acc, const double* __restrict__ part, int64_t ld,
                                                     int64_t p0, int64_t p1) {
    int64_t p = p0;
    for (; p + 8 <= p1; p += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(p + u) * ld];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; p < p1; ++p) acc += part[p * ld];
    return acc;
}

// rows of owners with several segments: G[a, :] = (accumulate ? G[a, :] : 0) + sum part
__global__ void k_seg_reduce_rows(SegDev sg, const double* __restrict__ part, int64_t q,
                                  double* __restrict__ G, int64_t ldg, int accumulate) {
    const int64_t o = blockIdx.x;
    const int64_t c = static_cast<int64_t>(blockIdx.y) * blockDim.x + threadIdx.x;
    if (o >= sg.nmulti || c >= q) return;
    const int64_t a = sg.multi_owner[o];
    double acc = accumulate ? G[a * ldg + c] : 0.0;
    acc = sum_parts_in_order(acc, part + c, q, sg.multi_ptr[o], sg.multi_ptr[o + 1]);
    G[a * ldg + c] = acc;
}

void launch_sparse_gram(const SegDev& sg, const int* rowidx, const double* cval,
                        const int64_t* rowptr, const int* colidx, const double* rval, int64_t q,
                        double* G, int64_t ldg, bool accumulate, double* part, hipStream_t st) {
    if (q <= 0 || sg.nseg <= 0) return;
    const int64_t chunk = std::min<int64_t>(q, 2048);
    const int64_t tasks = sg.nseg * ((q + chunk - 1) / chunk);
    const size_t lds = static_cast<size_t>(SG_WAVES) * chunk * sizeof(double);
    hipLaunchKernelGGL(k_sparse_gram, dim3(static_cast<unsigned>((tasks + SG_WAVES - 1) / SG_WAVES)),
                       dim3(SG_WAVES * 64), lds, st, sg, rowidx, cval, rowptr, colidx, rval, q,
                       chunk, G, ldg, accumulate ? 1 : 0, part);
    if (sg.nmulti > 0)
        hipLaunchKernelGGL(k_seg_reduce_rows, dim3(static_cast<unsigned>(sg.nmulti),
                                                   static_cast<unsigned>((q + 255) / 256)),
                           dim3(256), 0, st, sg, part, q, G, ldg, accumulate ? 1 : 0);
}

// P[:, a] = sigma .* (U^T S[:, a]) for a sparse S (CSC segments) and row-major U (rows x s),
// written into G at G[k, off + a] and mirrored at G[off + a, k].
__global__ __launch_bounds__(256) void k_sparse_proj(SegDev sg, const int* __restrict__ rowidx,
                                                     const double* __restrict__ cval,
                                                     const double* __restrict__ U, int64_t s,
                                                     const double* __restrict__ sigma,
                                                     double* __restrict__ G, int64_t ldg, int64_t off,
                                                     double* __restrict__ part) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t seg = static_cast<int64_t>(blockIdx.x) * 4 + wave;
    if (seg >= sg.nseg) return;
    const int64_t a = sg.owner[seg];
    const int pidx = sg.pidx[seg];
    const int64_t eb = sg.begin[seg], ee = sg.end[seg];
    for (int64_t k0 = 0; k0 < s; k0 += 8 * kWave) {
        double acc[8] = {};
        for (int64_t e = eb; e < ee; ++e) {
            const int64_t h = rowidx[e];
            const double v = cval[e];
            const double* Uh = U + h * s;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t k = k0 + u * kWave + lane;
                if (k < s) acc[u] += v * Uh[k];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t k = k0 + u * kWave + lane;
            if (k >= s) continue;
            if (pidx < 0) {
                const double val = acc[u] * sigma[k];
                G[k * ldg + off + a] = val;
                G[(off + a) * ldg + k] = val;
            } else {
                part[static_cast<int64_t>(pidx) * s + k] = acc[u];
            }
        }
    }
}

__global__ void k_seg_reduce_proj(SegDev sg, const double* __restrict__ part, int64_t s,
                                  const double* __restrict__ sigma, double* __restrict__ G,
                                  int64_t ldg, int64_t off) {
    const int64_t o = blockIdx.x;
    const int64_t k = static_cast<int64_t>(blockIdx.y) * blockDim.x + threadIdx.x;
    if (o >= sg.nmulti || k >= s) return;
    const int64_t a = sg.multi_owner[o];
    double acc = 0;
    acc = sum_parts_in_order(acc, part + k, s, sg.multi_ptr[o], sg.multi_ptr[o + 1]);
    const double val = acc * sigma[k];
    G[k * ldg + off + a] = val;
    G[(off + a) * ldg + k] = val;
}

void launch_sparse_proj(const SegDev& sg, const int* rowidx, const double* cval, const double* U,
                        int64_t s, const double* sigma, double* G, int64_t ldg, int64_t off,
                        double* part, hipStream_t st) {
    if (sg.nseg <= 0 || s <= 0) return;
    hipLaunchKernelGGL(k_sparse_proj, dim3(static_cast<unsigned>((sg.nseg + 3) / 4)), dim3(256), 0, st,
                       sg, rowidx, cval, U, s, sigma, G, ldg, off, part);
    if (sg.nmulti > 0)
        hipLaunchKernelGGL(k_seg_reduce_proj, dim3(static_cast<unsigned>(sg.nmulti),
                                                   static_cast<unsigned>((s + 255) / 256)),
                           dim3(256), 0, st, sg, part, s, sigma, G, ldg, off);
}

// C[crow(h), :] (+)= cs .* (S[h, :] B) for a sparse S (CSR segments over its rows) and a
// row-major B (K x N).
__global__ __launch_bounds__(256) void k_spmm_rows(SegDev sg, const int* __restrict__ colidx,
                                                   const double* __restrict__ rval,
                                                   const double* __restrict__ B, int64_t N,
                                                   const double* __restrict__ cs,
                                                   double* __restrict__ C, int64_t ldc,
                                                   const int* __restrict__ crow, int accumulate,
                                                   double* __restrict__ part) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t seg = static_cast<int64_t>(blockIdx.x) * 4 + wave;
    if (seg >= sg.nseg) return;
    const int64_t h = sg.owner[seg];
    const int pidx = sg.pidx[seg];
    const int64_t ci = crow ? crow[h] : h;
    double* Crow = C + ci * ldc;
    const int64_t eb = sg.begin[seg], ee = sg.end[seg];
    for (int64_t k0 = 0; k0 < N; k0 += 8 * kWave) {
        double acc[8] = {};
        for (int64_t e = eb; e < ee; ++e) {
            const double v = rval[e];
            const double* Bb = B + static_cast<int64_t>(colidx[e]) * N;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t k = k0 + u * kWave + lane;
                if (k < N) acc[u] += v * Bb[k];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t k = k0 + u * kWave + lane;
            if (k >= N) continue;
            if (pidx < 0) {
                double val = acc[u];
                if (cs) val *= cs[k];
                Crow[k] = accumulate ? Crow[k] + val : val;
            } else {
                part[static_cast<int64_t>(pidx) * N + k] = acc[u];
            }
        }
    }
}

__global__ void k_seg_reduce_spmm(SegDev sg, const double* __restrict__ part, int64_t N,
                                  const double* __restrict__ cs, double* __restrict__ C,
                                  int64_t ldc, const int* __restrict__ crow, int accumulate) {
    const int64_t o = blockIdx.x;
    const int64_t k = static_cast<int64_t>(blockIdx.y) * blockDim.x + threadIdx.x;
    if (o >= sg.nmulti || k >= N) return;
    const int64_t h = sg.multi_owner[o];
    double acc = 0;
    acc = sum_parts_in_order(acc, part + k, N, sg.multi_ptr[o], sg.multi_ptr[o + 1]);
    if (cs) acc *= cs[k];
    const int64_t ci = crow ? crow[h] : h;
    double* dst = C + ci * ldc + k;
    *dst = accumulate ? *dst + acc : acc;
}

void launch_spmm_rows(const SegDev& sg, const int* colidx, const double* rval, const double* B,
                      int64_t N, const double* cs, double* C, int64_t ldc, const int* crow,
                      bool accumulate, double* part, hipStream_t st, KernelTimer* timer) {
    if (sg.nseg <= 0 || N <= 0) return;
    FASTPI_LAUNCH(timer, KT_LABEL_SPMM, k_spmm_rows, dim3(static_cast<unsigned>((sg.nseg + 3) / 4)), dim3(256), 0,
                  st, sg, colidx, rval, B, N, cs, C, ldc, crow, accumulate ? 1 : 0, part);
    if (sg.nmulti > 0)
        FASTPI_LAUNCH(timer, KT_LABEL_SPMM, k_seg_reduce_spmm,
                      dim3(static_cast<unsigned>(sg.nmulti), static_cast<unsigned>((N + 255) / 256)), dim3(256),
                      0, st, sg, part, N, cs, C, ldc, crow, accumulate ? 1 : 0);
}

// Diagonal blocks of V1 Sigma1^2 V1^T into G2 (n1 x n1): one workgroup per dense block.
__global__ __launch_bounds__(256) void k_blockdiag_gram(const BlockWork* __restrict__ work,
                                                        const double* __restrict__ V1,
                                                        const double* __restrict__ sig1,
                                                        double* __restrict__ G, int64_t ldg) {
    const BlockWork w = work[blockIdx.x];
    const int nb = w.cols, sb = w.rank;
    const double* Vb = V1 + w.v_off;   // nb x sb, column-major
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        const int a = e / nb, b = e % nb;
        double acc = 0;
        for (int k = 0; k < sb; ++k) {
            const double sk = sig1[w.sig_off + k];
            acc += Vb[static_cast<int64_t>(k) * nb + a] * (sk * sk) * Vb[static_cast<int64_t>(k) * nb + b];
        }
        G[static_cast<int64_t>(w.col0 + a) * ldg + w.col0 + b] = acc;
    }
}

void launch_blockdiag_gram(const BlockWork* work, int nwork, const double* V1, const double* sig1,
                           double* G, int64_t ldg, hipStream_t st) {
    if (nwork <= 0) return;
    hipLaunchKernelGGL(k_blockdiag_gram, dim3(nwork), dim3(256), 0, st, work, V1, sig1, G, ldg);
}

// Top rows of U2 (Eq. 2): for block i, U2[row0 + r, :] = U_i[r, :] (Sigma_i V_i^T V2[col0:, :]
// Sigma2^-1). The KC x S_CH intermediate lives in LDS; the block rank runs in chunks of KC
// and the columns of U2 in chunks of S_CH.
constexpr int S_CH = 128;
constexpr int KC = 32;
constexpr int U2_UNROLL = 8;   // terms of a dot product whose loads are issued together
constexpr int U2_TASKS = 8;    // outputs of U2 a thread sums at once
constexpr int U2_KSTEP = 4;    // terms of each of them loaded together
__global__ __launch_bounds__(256) void k_u2_top(const BlockWork* __restrict__ work,
                                                const double* __restrict__ U1,
                                                const double* __restrict__ sig1,
                                                const double* __restrict__ V1,
                                                const double* __restrict__ V2, int64_t s,
                                                const double* __restrict__ inv_sig2,
                                                double* __restrict__ U2, int* status) {
    __shared__ double Tm[KC][S_CH + 1];
    const BlockWork w = work[blockIdx.x];
    const int mb = w.rows, nb = w.cols, sb = w.rank;
    (void)status;
    const double* Ub = U1 + w.u_off;   // mb x sb col-major
    const double* Vb = V1 + w.v_off;   // nb x sb col-major
    for (int64_t c0 = 0; c0 < s; c0 += S_CH) {
        const int nc = static_cast<int>(min<int64_t>(S_CH, s - c0));
        for (int k0 = 0; k0 < sb || k0 == 0; k0 += KC) {
            const int kc = min(KC, sb - k0);
            for (int e = threadIdx.x; e < kc * nc; e += blockDim.x) {
                const int k = e / nc, c = e % nc;
                const double* x = Vb + static_cast<int64_t>(k0 + k) * nb;
                const double* y = V2 + static_cast<int64_t>(w.col0) * s + c0 + c;
                // the sum in order over a; U2_UNROLL terms' loads in flight together
                double acc = 0;
                int a = 0;
                for (; a + U2_UNROLL <= nb; a += U2_UNROLL) {
                    double xv[U2_UNROLL], yv[U2_UNROLL];
#pragma unroll
                    for (int u = 0; u < U2_UNROLL; ++u) {
                        xv[u] = x[a + u];
                        yv[u] = y[static_cast<int64_t>(a + u) * s];
                    }
#pragma unroll
                    for (int u = 0; u < U2_UNROLL; ++u) acc += xv[u] * yv[u];
                }
                for (; a < nb; ++a) acc += x[a] * y[static_cast<int64_t>(a) * s];
                Tm[k][c] = acc * sig1[w.sig_off + k0 + k] * inv_sig2[c0 + c];
            }
            __syncthreads();
            // U2_TASKS outputs per thread at a time, each summed in order over k, with the
            // loads of U2_TASKS x U2_KSTEP terms in flight together
            const int ntask = mb * nc;
            for (int e0 = threadIdx.x; e0 < ntask; e0 += U2_TASKS * static_cast<int>(blockDim.x)) {
                int rr[U2_TASKS], cc[U2_TASKS];
                double acc[U2_TASKS];
#pragma unroll
                for (int j = 0; j < U2_TASKS; ++j) {
                    const int e = min(e0 + j * static_cast<int>(blockDim.x), ntask - 1);
                    rr[j] = e / nc;
                    cc[j] = e % nc;
                    acc[j] = 0.0;
                }
                const double* ub = Ub + static_cast<int64_t>(k0) * mb;
                int k = 0;
                for (; k + U2_KSTEP <= kc; k += U2_KSTEP) {
                    double uv[U2_TASKS][U2_KSTEP];
#pragma unroll
                    for (int j = 0; j < U2_TASKS; ++j)
#pragma unroll
                        for (int u = 0; u < U2_KSTEP; ++u) uv[j][u] = ub[static_cast<int64_t>(k + u) * mb + rr[j]];
#pragma unroll
                    for (int j = 0; j < U2_TASKS; ++j)
#pragma unroll
                        for (int u = 0; u < U2_KSTEP; ++u) acc[j] += uv[j][u] * Tm[k + u][cc[j]];
                }
                for (; k < kc; ++k) {
                    double uv[U2_TASKS];
#pragma unroll
                    for (int j = 0; j < U2_TASKS; ++j) uv[j] = ub[static_cast<int64_t>(k) * mb + rr[j]];
#pragma unroll
                    for (int j = 0; j < U2_TASKS; ++j) acc[j] += uv[j] * Tm[k][cc[j]];
                }
#pragma unroll
                for (int j = 0; j < U2_TASKS; ++j) {
                    if (e0 + j * static_cast<int>(blockDim.x) >= ntask) break;
                    double* dst = U2 + static_cast<int64_t>(w.row0 + rr[j]) * s + c0 + cc[j];
                    *dst = k0 == 0 ? acc[j] : *dst + acc[j];
                }
            }
            __syncthreads();
            if (sb == 0) break;
        }
    }
}

void launch_u2_top(const BlockWork* work, int nwork, const double* U1, const double* sig1,
                   const double* V1, const double* V2, int64_t s, const double* inv_sig2,
                   double* U2, int* status, hipStream_t st) {
    if (nwork <= 0 || s <= 0) return;
    hipLaunchKernelGGL(k_u2_top, dim3(nwork), dim3(256), 0, st, work, U1, sig1, V1, V2, s, inv_sig2,
                       U2, status);
}

// sigma = sqrt(max(lam, 0)); inv = 1/sigma above the cut-off (else 0) -- for the rank
// deficient case the corresponding columns are zero (their singular value is 0 in effect)
// sigma = sqrt(lambda) and its reciprocal for the t kept eigenvalues of a Gram matrix; a
// value at or below rel_cut times the largest is not resolved by the Gram matrix and is
// returned as 0 (reciprocal 0), with bit 8 of the owner's status word set when the largest
// is positive (the kept rank reaches the floor)
__global__ void k_sqrt_inv(const double* __restrict__ lam, int64_t t, double rel_cut,
                           double* __restrict__ sigma, double* __restrict__ inv, int* __restrict__ status) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= t) return;
    const double l0 = lam[0] > 0 ? lam[0] : 0.0;
    const double l = lam[k] > 0 ? lam[k] : 0.0;
    const double sg = sqrt(l);
    const bool keep = sg > rel_cut * sqrt(l0);
    sigma[k] = keep ? sg : 0.0;
    inv[k] = keep ? 1.0 / sg : 0.0;
    if (!keep && l0 > 0 && status) atomicOr(status, kStatusFloor);
}

void launch_sqrt_inv(const double* lam, int64_t t, double rel_cut, double* sigma, double* inv, int* status,
                     hipStream_t st) {
    if (t <= 0) return;
    hipLaunchKernelGGL(k_sqrt_inv, dim3(static_cast<unsigned>((t + 255) / 256)), dim3(256), 0, st, lam, t,
                       rel_cut, sigma, inv, status);
}

// C1 = diag(sig2) Vt[0:s, :] diag(inv3) (s x r) and C2 = Vt[s:, :] diag(inv3) (n2 x r)
__global__ void k_col_coeffs(const double* __restrict__ Vt, int64_t s, int64_t n2, int64_t r,
                             const double* __restrict__ sig2, const double* __restrict__ inv3,
                             double* __restrict__ C1, double* __restrict__ C2) {
    const int64_t n = (s + n2) * r;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int64_t i = e / r, k = e % r;
        const double v = Vt[e] * inv3[k];
        if (i < s) C1[i * r + k] = v * sig2[i];
        else C2[(i - s) * r + k] = v;
    }
}

void launch_col_coeffs(const double* Vt, int64_t s, int64_t n2, int64_t r, const double* sig2,
                       const double* inv3, double* C1, double* C2, hipStream_t st) {
    const int64_t n = (s + n2) * r;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_col_coeffs, dim3(static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 8192))),
                       dim3(256), 0, st, Vt, s, n2, r, sig2, inv3, C1, C2);
}

// V rows of the hub columns: V[invF[n1 + j], :] = Vt[s + j, :]
__global__ void k_copy_rows(const double* __restrict__ src, int64_t rows, int64_t cols,
                            const int* __restrict__ dst_row, double* __restrict__ dst) {
    const int64_t n = rows * cols;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int64_t i = e / cols, k = e % cols;
        dst[static_cast<int64_t>(dst_row[i]) * cols + k] = src[e];
    }
}

void launch_copy_rows(const double* src, int64_t rows, int64_t cols, const int* dst_row, double* dst,
                      hipStream_t st) {
    const int64_t n = rows * cols;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy_rows, dim3(static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 8192))),
                       dim3(256), 0, st, src, rows, cols, dst_row, dst);
}

// S^+ for the apply: inv[k] = 1/S[k] if S[k] > cut * max(S) else 0
__global__ void k_pinv_sigma(const double* __restrict__ S, int64_t r, double cut,
                             double* __restrict__ inv) {
    __shared__ double smax;
    if (threadIdx.x == 0) {
        double mx = 0;
        for (int64_t k = 0; k < r; ++k) mx = S[k] > mx ? S[k] : mx;
        smax = mx;
    }
    __syncthreads();
    for (int64_t k = threadIdx.x; k < r; k += blockDim.x) {
        const double v = S[k];
        inv[k] = v > cut * smax ? 1.0 / v : 0.0;
    }
}

void launch_pinv_sigma(const double* S, int64_t r, double cut, double* inv, hipStream_t st) {
    if (r <= 0) return;
    hipLaunchKernelGGL(k_pinv_sigma, dim3(1), dim3(256), 0, st, S, r, cut, inv);
}

}  // namespace fastpi
