// Planner: reordering, per-block ranks (Eq. 1), stage ranks (Eqs. 2-3) and the index maps
// that move the caller's CSR values into the device layout. Host only; integer work.
#include <algorithm>
#include <numeric>

#include "host_internal.h"

namespace fastpi {

void build_segments(const std::vector<int64_t>& ptr, Segments& out) {
    out = Segments{};
    const int64_t owners = static_cast<int64_t>(ptr.size()) - 1;
    out.multi_ptr.push_back(0);
    for (int64_t o = 0; o < owners; ++o) {
        const int64_t b = ptr[o], e = ptr[o + 1];
        if (e <= b) continue;
        const int64_t nseg = (e - b + kSegLen - 1) / kSegLen;
        for (int64_t k = 0; k < nseg; ++k) {
            out.owner.push_back(static_cast<int32_t>(o));
            out.begin.push_back(b + k * kSegLen);
            out.end.push_back(std::min(e, b + (k + 1) * kSegLen));
            out.pidx.push_back(nseg > 1 ? static_cast<int32_t>(out.npart++) : -1);
        }
        if (nseg > 1) {
            out.multi_owner.push_back(static_cast<int32_t>(o));
            out.multi_ptr.push_back(static_cast<int32_t>(out.npart));
        }
    }
}

// Block work list, packed-output offsets and stage ranks for the given per-block ranks:
// s = min(ceil(alpha n1), s_b + m2, n1) and r = min(ceil(alpha min(m, n)), s + n2, m).
void assign_ranks(Plan& p, const std::vector<int64_t>& ranks) {
    const ReorderOut& R = p.ro;
    const int64_t B = static_cast<int64_t>(R.blocks.size());
    p.block_rank.assign(B, 0);
    p.work.clear();
    int64_t blk = 0, u1 = 0, v1 = 0, sb = 0;
    for (int64_t b = 0; b < B; ++b) {
        const BlockDesc& d = R.blocks[b];
        if (d.rows == 0 || d.cols == 0) continue;
        const int64_t si = std::max<int64_t>(0, std::min({ranks[b], d.rows, d.cols}));
        p.block_rank[b] = si;
        BlockWork w{};
        w.data_off = blk;
        w.u_off = u1;
        w.v_off = v1;
        w.rows = static_cast<int32_t>(d.rows);
        w.cols = static_cast<int32_t>(d.cols);
        w.rank = static_cast<int32_t>(si);
        w.sig_off = static_cast<int32_t>(sb);
        w.row0 = static_cast<int32_t>(d.row0);
        w.col0 = static_cast<int32_t>(d.col0);
        p.work.push_back(w);
        blk += d.rows * d.cols;
        u1 += d.rows * si;
        v1 += d.cols * si;
        sb += si;
    }
    p.B_dense = static_cast<int64_t>(p.work.size());
    p.blk_elems = blk;
    p.u1_elems = u1;
    p.v1_elems = v1;
    p.s_b = sb;
    p.s = std::min({target_rank(p.alpha, R.n1), sb + R.m2, R.n1});
    p.r = std::min({target_rank(p.alpha, std::min(p.m, p.n)), p.s + R.n2, p.m});
    // largest Jacobi cost first (p q^2 with p >= q), ties by block order
    std::stable_sort(p.work.begin(), p.work.end(), [](const BlockWork& a, const BlockWork& b) {
        auto cost = [](const BlockWork& w) {
            const int64_t pp = std::max(w.rows, w.cols), qq = std::min(w.rows, w.cols);
            return pp * qq * qq;
        };
        return cost(a) > cost(b);
    });
}

int block_features(const Plan& p, const double* val, double* out) {
    const ReorderOut& R = p.ro;
    // dense blocks rebuilt from the value maps (block order, column-major per block)
    std::vector<double> blk(static_cast<size_t>(p.blk_elems), 0.0);
    for (int64_t e = 0; e < p.nnz; ++e)
        if (p.dst0[e] >= 0 && p.dst0[e] < p.blk_elems) blk[p.dst0[e]] = val[e];
    double a11 = 0;
    for (double v : blk) a11 += v * v;
    const double tiny = 1e-300;
    const int64_t B = static_cast<int64_t>(R.blocks.size());
    int64_t off = 0, k = 0;
    for (int64_t b = 0; b < B; ++b) {
        const BlockDesc& d = R.blocks[b];
        if (d.rows == 0 || d.cols == 0) continue;
        const int64_t mi = d.rows, ni = d.cols;
        const double* A = blk.data() + off;
        int64_t nnz = 0;
        double fro2 = 0, cmax = 0, cmin = 0, lsum = 0, rmax = 0;
        std::vector<double> lc(ni), row2(mi, 0.0);
        for (int64_t c = 0; c < ni; ++c) {
            double s = 0;
            for (int64_t r = 0; r < mi; ++r) {
                const double v = A[c * mi + r];
                nnz += (v != 0.0);
                s += v * v;
                row2[r] += v * v;
            }
            fro2 += s;
            cmax = c == 0 ? s : std::max(cmax, s);
            cmin = c == 0 ? s : std::min(cmin, s);
            lc[c] = std::log(std::max(s, tiny));
            lsum += lc[c];
        }
        for (int64_t r = 0; r < mi; ++r) rmax = std::max(rmax, row2[r]);
        const double lmean = lsum / static_cast<double>(ni);
        double var = 0;
        for (int64_t c = 0; c < ni; ++c) var += (lc[c] - lmean) * (lc[c] - lmean);
        var /= static_cast<double>(ni);
        int64_t hub = 0;
        for (int64_t r = d.row0; r < d.row0 + mi; ++r) hub += p.t_rowptr[r + 1] - p.t_rowptr[r];
        for (int64_t c = d.col0; c < d.col0 + ni; ++c) hub += p.a21_colptr[c + 1] - p.a21_colptr[c];
        double* f = out + k * 16;
        f[0] = std::log(static_cast<double>(mi));
        f[1] = std::log(static_cast<double>(ni));
        f[2] = std::log(static_cast<double>(std::max<int64_t>(nnz, 1)));
        f[3] = static_cast<double>(nnz) / static_cast<double>(mi * ni);
        f[4] = std::log(std::max(fro2, tiny));
        f[5] = std::log(std::max(cmax, tiny));
        f[6] = std::log(std::max(cmin, tiny));
        f[7] = lmean;
        f[8] = std::sqrt(var);
        f[9] = std::log(std::max(rmax, tiny));
        f[10] = fro2 / std::max(cmax, tiny);
        f[11] = fro2 / std::max(a11, tiny);
        f[12] = p.alpha;
        f[13] = static_cast<double>(ni) / static_cast<double>(std::max<int64_t>(R.n1, 1));
        f[14] = std::log1p(static_cast<double>(hub));
        f[15] = static_cast<double>(b) / static_cast<double>(std::max<int64_t>(B, 1));
        off += mi * ni;
        ++k;
    }
    return FASTPI_OK;
}

int build_plan(Plan& p, int64_t m, int64_t n, const int64_t* rowptr, const int32_t* col,
               const double* val, double alpha, double k, const ReorderOut* given) {
    if (!(alpha > 0.0 && alpha <= 1.0)) {
        set_error("alpha must lie in (0, 1]");
        return FASTPI_EINVAL;
    }
    int st = validate_csr(m, n, rowptr, col, val);
    if (st != FASTPI_OK) return st;
    if (given) {
        p.ro = *given;
    } else {
        st = reorder_pattern(m, n, rowptr, col, val, k, p.ro);
        if (st != FASTPI_OK) return st;
    }
    p.m = m;
    p.n = n;
    p.nnz = rowptr[m];
    p.alpha = alpha;
    p.k = k;
    const ReorderOut& R = p.ro;
    const int64_t m1 = R.m1, n1 = R.n1, m2 = R.m2, n2 = R.n2;
    const int64_t B = static_cast<int64_t>(R.blocks.size());

    std::vector<int64_t> ranks(B, 0);
    for (int64_t b = 0; b < B; ++b) {
        const BlockDesc& d = R.blocks[b];
        if (d.rows > 0 && d.cols > 0) ranks[b] = std::min({target_rank(alpha, d.cols), d.rows, d.cols});
    }
    assign_ranks(p, ranks);

    // inverse permutations and the block id of every spoke row
    p.invT.assign(m, 0);
    p.invF.assign(n, 0);
    for (int64_t i = 0; i < m; ++i) p.invT[R.piT[i]] = static_cast<int32_t>(i);
    for (int64_t j = 0; j < n; ++j) p.invF[R.piF[j]] = static_cast<int32_t>(j);
    std::vector<int64_t> row_blk(m1, -1), blk_data(B, -1);
    for (int64_t b = 0; b < B; ++b) {
        const BlockDesc& d = R.blocks[b];
        for (int64_t i = d.row0; i < d.row0 + d.rows; ++i) row_blk[i] = b;
    }
    {
        int64_t off = 0;
        for (int64_t b = 0; b < B; ++b) {
            const BlockDesc& d = R.blocks[b];
            if (d.rows == 0 || d.cols == 0) continue;
            blk_data[b] = off;
            off += d.rows * d.cols;
        }
    }

    // count A21 and T entries per row / column (new ids), skipping stored zeros
    const int64_t nnz = rowptr[m];
    p.dst0.assign(nnz, -1);
    p.dst1.assign(nnz, -1);
    p.a21_rowptr.assign(m2 + 1, 0);
    p.a21_colptr.assign(n1 + 1, 0);
    p.t_rowptr.assign(m + 1, 0);
    p.t_colptr.assign(n2 + 1, 0);
    for (int64_t i = 0; i < m; ++i) {
        const int64_t ni = R.piT[i];
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (val && val[e] == 0.0) continue;
            const int64_t nj = R.piF[col[e]];
            if (nj >= n1) {
                p.t_rowptr[ni + 1]++;
                p.t_colptr[nj - n1 + 1]++;
            } else if (ni >= m1) {
                p.a21_rowptr[ni - m1 + 1]++;
                p.a21_colptr[nj + 1]++;
            }
        }
    }
    for (int64_t i = 0; i < m2; ++i) p.a21_rowptr[i + 1] += p.a21_rowptr[i];
    for (int64_t j = 0; j < n1; ++j) p.a21_colptr[j + 1] += p.a21_colptr[j];
    for (int64_t i = 0; i < m; ++i) p.t_rowptr[i + 1] += p.t_rowptr[i];
    for (int64_t j = 0; j < n2; ++j) p.t_colptr[j + 1] += p.t_colptr[j];
    const int64_t nnz21 = p.a21_rowptr[m2], nnzT = p.t_rowptr[m];
    p.off_a21r = p.blk_elems;
    p.off_a21c = p.off_a21r + nnz21;
    p.off_tr = p.off_a21c + nnz21;
    p.off_tc = p.off_tr + nnzT;
    p.val_elems = p.off_tc + nnzT;
    p.a21_colidx.assign(nnz21, 0);
    p.a21_rowidx.assign(nnz21, 0);
    p.t_colidx.assign(nnzT, 0);
    p.t_rowidx.assign(nnzT, 0);

    // Row-major fill: visiting new rows in ascending order and, inside a row, columns in
    // ascending new id gives sorted CSR rows; the CSC fill in the same visiting order gives
    // ascending row ids inside every column.
    std::vector<int64_t> fill21r(p.a21_rowptr.begin(), p.a21_rowptr.end() - 1);
    std::vector<int64_t> fill21c(p.a21_colptr.begin(), p.a21_colptr.end() - 1);
    std::vector<int64_t> filltr(p.t_rowptr.begin(), p.t_rowptr.end() - 1);
    std::vector<int64_t> filltc(p.t_colptr.begin(), p.t_colptr.end() - 1);
    std::vector<std::pair<int32_t, int64_t>> rowbuf;
    for (int64_t ni = 0; ni < m; ++ni) {
        const int64_t i = p.invT[ni];
        rowbuf.clear();
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (val && val[e] == 0.0) continue;
            rowbuf.emplace_back(R.piF[col[e]], e);
        }
        std::sort(rowbuf.begin(), rowbuf.end());
        for (const auto& pr : rowbuf) {
            const int64_t nj = pr.first, e = pr.second;
            if (nj >= n1) {
                const int64_t tr = filltr[ni]++, tc = filltc[nj - n1]++;
                p.t_colidx[tr] = static_cast<int32_t>(nj - n1);
                p.t_rowidx[tc] = static_cast<int32_t>(ni);
                p.dst0[e] = p.off_tr + tr;
                p.dst1[e] = p.off_tc + tc;
            } else if (ni >= m1) {
                const int64_t ar = fill21r[ni - m1]++, ac = fill21c[nj]++;
                p.a21_colidx[ar] = static_cast<int32_t>(nj);
                p.a21_rowidx[ac] = static_cast<int32_t>(ni - m1);
                p.dst0[e] = p.off_a21r + ar;
                p.dst1[e] = p.off_a21c + ac;
            } else {
                const int64_t b = row_blk[ni];
                const BlockDesc& d = R.blocks[b];
                if (b < 0 || nj < d.col0 || nj >= d.col0 + d.cols) {
                    set_error("internal: A11 entry outside its diagonal block");
                    return FASTPI_EINTERNAL;
                }
                p.dst0[e] = blk_data[b] + (nj - d.col0) * d.rows + (ni - d.row0);
            }
        }
    }
    build_segments(p.a21_colptr, p.seg_a21c);
    build_segments(p.a21_rowptr, p.seg_a21r);
    build_segments(p.t_colptr, p.seg_tc);
    build_segments(p.t_rowptr, p.seg_tr);
    return FASTPI_OK;
}

}  // namespace fastpi
