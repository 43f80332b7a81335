// host_csr.cpp -- host-only logic of the library: parameter defaults,
// Algorithm 1's level schedule, CSR validation, the transpose check and the
// row-length binning of a CSR matrix into workgroup row blocks.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <thread>

#include "internal.h"

namespace {

void put_msg(char *msg, int len, const char *text) {
    if (msg && len > 0) {
        std::snprintf(msg, (size_t)len, "%s", text);
    }
}

}  // namespace

extern "C" int pdhg_params_default(pdhg_params *p) {
    if (!p) return PDHG_E_ARG;
    std::memset(p, 0, sizeof(*p));
    p->precision = PDHG_FP64;
    p->ruiz_passes = 10;
    p->power_iters = 100;
    p->eval_every = 64;
    p->literal_snapshots = 0;
    p->n_levels = 0;
    p->levels = nullptr;
    p->eps_rel = 1e-6;
    p->eta = 0.0;
    p->omega0 = 0.0;
    p->eta_factor = 0.9;
    p->beta_suff = 0.2;
    p->beta_nec = 0.8;
    p->beta_art = 0.36;
    p->omega_theta = 0.5;
    p->max_iters = (int64_t)1 << 62;
    p->time_limit_s = 3600.0;
    p->use_graph = 1;
    p->variant = 0;
    p->reflect = 1.0;
    p->omega_rule = 0;
    p->pid_kp = 0.99;
    p->pid_ki = 0.01;
    p->pid_kd = 0.0;
    p->stop_on = 0;
    p->polish = 0;
    p->polish_frac = 0.125;
    return PDHG_OK;
}

extern "C" int pdhg_refine_params_default(pdhg_refine_params *p) {
    if (!p) return PDHG_E_ARG;
    std::memset(p, 0, sizeof(*p));
    p->outer_eps = 1e-8;
    p->inner_eps = 1e-4;
    p->max_rounds = 8;
    p->cap_log2 = 10;
    p->max_inner_iters = 200000;
    p->progress = 1e-2;
    p->inner_precision = PDHG_FP32;
    p->omega_carry = 1;
    return PDHG_OK;
}

// Algorithm 1 (Section 3.1) lowers its target tenfold after every launch,
// starting at eps_cross, and stops PDHG at eps_rel.  The levels are formed
// as eps_cross / 10^j so that rounding cannot leave a level a hair above
// eps_rel (repeated multiplication by 0.1 does).
extern "C" int pdhg_alg1_levels(double eps_cross, double eps_rel, double *out,
                                int cap) {
    if (!out || cap < 1 || !(eps_cross > 0.0) || !(eps_rel > 0.0))
        return PDHG_E_ARG;
    int k = 0;
    double p10 = 1.0;
    for (int j = 0; j < 64 && k < cap; ++j) {
        double lev = eps_cross / p10;
        p10 *= 10.0;
        if (lev <= eps_rel * (1.0 + 1e-9)) break;
        out[k++] = lev;
    }
    if (k < cap) out[k++] = eps_rel;
    return k;
}

extern "C" int pdhg_validate_csr(int64_t rows, int64_t cols, int64_t nnz,
                                 const int64_t *rp, const int32_t *ci,
                                 char *msg, int msg_len) {
    char buf[256];
    if (rows < 1 || cols < 1) {
        put_msg(msg, msg_len, "matrix must have at least one row and column");
        return PDHG_E_CSR;
    }
    if (nnz < 0 || nnz >= ((int64_t)1 << 31)) {
        put_msg(msg, msg_len, "nnz must be in [0, 2^31)");
        return PDHG_E_CSR;
    }
    if (cols >= ((int64_t)1 << 31) || rows >= ((int64_t)1 << 31)) {
        put_msg(msg, msg_len, "dimensions must be below 2^31");
        return PDHG_E_CSR;
    }
    if (!rp || (nnz > 0 && !ci)) {
        put_msg(msg, msg_len, "null CSR array");
        return PDHG_E_CSR;
    }
    if (rp[0] != 0 || rp[rows] != nnz) {
        std::snprintf(buf, sizeof buf,
                      "row pointers must start at 0 and end at nnz=%lld "
                      "(got %lld..%lld)",
                      (long long)nnz, (long long)rp[0], (long long)rp[rows]);
        put_msg(msg, msg_len, buf);
        return PDHG_E_CSR;
    }
    for (int64_t i = 0; i < rows; ++i) {
        if (rp[i + 1] < rp[i]) {
            std::snprintf(buf, sizeof buf, "row pointers decrease at row %lld",
                          (long long)i);
            put_msg(msg, msg_len, buf);
            return PDHG_E_CSR;
        }
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= cols) {
                std::snprintf(buf, sizeof buf,
                              "column index %d out of range in row %lld",
                              ci[p], (long long)i);
                put_msg(msg, msg_len, buf);
                return PDHG_E_CSR;
            }
            if (p > rp[i] && ci[p] <= ci[p - 1]) {
                std::snprintf(buf, sizeof buf,
                              "column indices not strictly increasing in "
                              "row %lld",
                              (long long)i);
                put_msg(msg, msg_len, buf);
                return PDHG_E_CSR;
            }
        }
    }
    return PDHG_OK;
}

// A^T's row j lists the rows i of A's column j in increasing order.  Walking
// A row by row and appending each (i, j) to a cursor per column therefore
// visits A^T's entries in storage order, which gives the permutation and
// the check in one O(nnz) pass.
extern "C" int pdhg_check_transpose(int64_t m, int64_t n, int64_t nnz,
                                    const int64_t *a_rp, const int32_t *a_ci,
                                    const double *a_v, const int64_t *at_rp,
                                    const int32_t *at_ci, const double *at_v,
                                    int64_t *perm, char *msg, int msg_len) {
    int rc = pdhg_validate_csr(m, n, nnz, a_rp, a_ci, msg, msg_len);
    if (rc != PDHG_OK) return rc;
    rc = pdhg_validate_csr(n, m, nnz, at_rp, at_ci, msg, msg_len);
    if (rc != PDHG_OK) return rc;
    if (nnz > 0 && (!a_v || !at_v)) {
        put_msg(msg, msg_len, "null value array");
        return PDHG_E_ARG;
    }
    std::vector<int64_t> cur(at_rp, at_rp + n);
    char buf[256];
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t p = a_rp[i]; p < a_rp[i + 1]; ++p) {
            int32_t j = a_ci[p];
            int64_t q = cur[j]++;
            if (q >= at_rp[j + 1] || at_ci[q] != (int32_t)i ||
                std::memcmp(&at_v[q], &a_v[p], sizeof(double)) != 0) {
                std::snprintf(buf, sizeof buf,
                              "A^T differs from the transpose of A at "
                              "A(%lld,%d)",
                              (long long)i, j);
                put_msg(msg, msg_len, buf);
                return PDHG_E_TRANSPOSE;
            }
            if (perm) perm[p] = q;
        }
    }
    for (int64_t j = 0; j < n; ++j) {
        if (cur[j] != at_rp[j + 1]) {
            std::snprintf(buf, sizeof buf,
                          "A^T row %lld has entries absent from A",
                          (long long)j);
            put_msg(msg, msg_len, buf);
            return PDHG_E_TRANSPOSE;
        }
    }
    return PDHG_OK;
}

extern "C" int pdhg_plan_bins(int64_t rows, const int64_t *rp, int tile,
                              int64_t split_threshold, int64_t split_chunk,
                              int32_t *out, int64_t cap) {
    if (rows < 1 || !rp || tile < 1 || split_chunk < 1 ||
        split_threshold < tile)
        return PDHG_E_ARG;
    pdhg::HostBins hb =
        pdhg::build_row_blocks(rows, rp, tile, split_threshold, split_chunk);
    const int64_t k = (int64_t)hb.blocks.size();
    for (int64_t i = 0; i < k && i < cap && out; ++i) {
        out[4 * i + 0] = hb.blocks[i].r0;
        out[4 * i + 1] = hb.blocks[i].r1;
        out[4 * i + 2] = hb.blocks[i].part;
        out[4 * i + 3] = hb.blocks[i].nparts;
    }
    return (int)k;
}

extern "C" int pdhg_choose_panels(int64_t rows, int64_t cols, int64_t nnz) {
    if (rows < 1 || cols < 1 || nnz < 0) return PDHG_E_ARG;
    return pdhg::choose_panels(rows, cols, nnz);
}

extern "C" int pdhg_plan_panels(int64_t rows, int64_t cols, const int64_t *rp,
                                const int32_t *ci, int P, const int64_t *cut,
                                int tile, int64_t *srp, int32_t *src,
                                int32_t *out, int64_t cap) {
    if (rows < 1 || cols < 1 || !rp || !cut || tile < 1 ||
        !(P == 1 || P == 2 || P == 4 || P == 8) || !srp || !src ||
        (int64_t)P * rows >= ((int64_t)1 << 31))
        return PDHG_E_ARG;
    if (rp[rows] > 0 && !ci) return PDHG_E_ARG;
    if (cut[0] != 0 || cut[P] != cols) return PDHG_E_ARG;
    for (int p = 0; p < P; ++p)
        if (cut[p + 1] < cut[p]) return PDHG_E_ARG;
    std::vector<int64_t> vc(cut, cut + P + 1);
    pdhg::Panels S = pdhg::build_panels(rows, rp, ci, P, vc);
    std::memcpy(srp, S.rp.data(), S.rp.size() * sizeof(int64_t));
    if (!S.src.empty())
        std::memcpy(src, S.src.data(), S.src.size() * sizeof(int32_t));
    pdhg::HostBins hb = pdhg::build_panel_blocks(rows, S.rp.data(), P, tile,
                                                 (int64_t)1 << 40, (int64_t)1 << 20);
    const int64_t k = (int64_t)hb.blocks.size();
    for (int64_t i = 0; i < k && i < cap && out; ++i) {
        out[4 * i + 0] = hb.blocks[i].r0;
        out[4 * i + 1] = hb.blocks[i].r1;
        out[4 * i + 2] = hb.blocks[i].part;
        out[4 * i + 3] = hb.blocks[i].nparts;
    }
    return (int)k;
}

namespace pdhg {

// Row-length bins.  Consecutive rows are packed into multi-row blocks of at
// most `tile` nonzeros (and at most `tile` rows); a row longer than `tile`
// gets a workgroup of its own, and a row longer than split_threshold is cut
// into parts of split_chunk nonzeros on several workgroups.  Single-row and
// split blocks are placed first so that the longest work starts first.
HostBins build_row_blocks(int64_t rows, const int64_t *rp, int tile,
                          int64_t split_threshold, int64_t split_chunk,
                          int max_rows, bool skip_empty) {
    HostBins hb;
    // rows per multi-row block: at most `tile`, and at most max_rows if set
    const int64_t row_cap = max_rows > 0 ? std::min<int64_t>(tile, max_rows) : tile;
    std::vector<RowBlock> longb, multi;
    std::vector<std::pair<int64_t, int64_t>> singles;  // (len, row)
    int slot = 0;
    int64_t r = 0;
    while (r < rows) {
        int64_t len = rp[r + 1] - rp[r];
        if (skip_empty && len == 0) {   // no block starts at an empty row
            ++r;
            continue;
        }
        if (len > tile) {
            if (len > split_threshold) {
                int nparts = (int)((len + split_chunk - 1) / split_chunk);
                for (int q = 0; q < nparts; ++q)
                    longb.push_back({(int32_t)r, (int32_t)(r + 1), q, nparts,
                                     slot, 0, 0, 0});
                hb.splits.push_back({(int32_t)r, nparts});
                hb.maxparts = std::max(hb.maxparts, nparts);
                hb.counts[2] += nparts;
                ++slot;
            } else {
                singles.push_back({len, r});
            }
            ++r;
            continue;
        }
        int64_t r1 = r, acc = 0;
        while (r1 < rows && (r1 - r) < row_cap) {
            int64_t l = rp[r1 + 1] - rp[r1];
            if (l > tile || acc + l > tile) break;
            acc += l;
            ++r1;
        }
        multi.push_back({(int32_t)r, (int32_t)r1, 0, 1, -1, 0, 0, 0});
        if (r1 - r == 1)
            hb.counts[1] += 1;
        else
            hb.counts[0] += 1;
        r = r1;
    }
    std::stable_sort(singles.begin(), singles.end(),
                     [](const std::pair<int64_t, int64_t> &a,
                        const std::pair<int64_t, int64_t> &b) {
                         return a.first > b.first;
                     });
    hb.blocks.reserve(longb.size() + singles.size() + multi.size());
    for (auto &b : longb) hb.blocks.push_back(b);
    for (auto &s : singles) {
        hb.blocks.push_back({(int32_t)s.second, (int32_t)(s.second + 1), 0, 1,
                             -1, 0, 0, 0});
        hb.counts[1] += 1;
    }
    for (auto &b : multi) hb.blocks.push_back(b);
    // nonzero range of each block, so that its loads need no row pointer
    for (auto &b : hb.blocks) {
        b.p0 = (int32_t)rp[b.r0];
        b.p1 = (int32_t)rp[b.r1];
    }
    return hb;
}

// Internal relabeling: rows of A and columns of A in order of decreasing
// length (stable).  With rows sorted, the row-length bins of both A and A^T
// are contiguous runs; with columns sorted, the most-referenced entries of x
// sit together, so on skewed matrices most gathers of x hit a small region
// that stays in cache.  A' keeps each row's entries sorted by the new column
// index; A'^T is built from A' by one pass with a cursor per column.
//
// A dimension split into P > 1 panels (column panels of the gather table of
// one SpMV side, see choose_panels) is dealt rather than sorted when it is
// skewed: rank r of the decreasing-length order goes to panel r % P, so every
// panel holds the same number of entries and the same share of long ones,
// each panel still in decreasing-length order.  Unskewed dimensions keep
// their order and are cut into P equal ranges.
static std::vector<int64_t> deal(std::vector<int32_t> &order, int P) {
    const int64_t k = (int64_t)order.size();
    std::vector<int64_t> cut((size_t)P + 1, 0);
    for (int p = 0; p < P; ++p) cut[p + 1] = cut[p] + (k - p + P - 1) / P;
    std::vector<int32_t> dealt((size_t)k);
    for (int64_t r = 0; r < k; ++r) dealt[cut[r % P] + r / P] = order[r];
    order.swap(dealt);
    return cut;
}

static std::vector<int64_t> even_cuts(int64_t k, int P) {
    std::vector<int64_t> cut((size_t)P + 1);
    for (int p = 0; p <= P; ++p) cut[p] = k * p / P;
    return cut;
}

Relabeled relabel(int64_t m, int64_t n, int64_t nnz, const int64_t *a_rp,
                  const int32_t *a_ci, const double *a_v,
                  const int64_t *at_rp, int panels_a, int panels_at,
                  int sort_rows, int sort_cols) {
    Relabeled R;
    R.pr.resize((size_t)m);
    R.pc.resize((size_t)n);
    std::iota(R.pr.begin(), R.pr.end(), 0);
    std::iota(R.pc.begin(), R.pc.end(), 0);
    // a dimension is reordered only when its lengths are skewed (longest
    // more than kSkew times the mean); otherwise its given order, which may
    // carry locality of its own, is kept
    auto skewed = [](const int64_t *rp, int64_t k) {
        int64_t mx = 0;
        for (int64_t i = 0; i < k; ++i) mx = std::max(mx, rp[i + 1] - rp[i]);
        return k > 0 && (double)mx > kSkew * (double)rp[k] / (double)k;
    };
    // sort_rows / sort_cols: -1 decides by skew, 0 keeps, 1 sorts
    R.sorted_rows = sort_rows < 0 ? skewed(a_rp, m) : sort_rows == 1;
    R.sorted_cols = sort_cols < 0 ? skewed(at_rp, n) : sort_cols == 1;
    if (R.sorted_rows)
        std::stable_sort(R.pr.begin(), R.pr.end(), [&](int32_t a, int32_t b) {
            return a_rp[a + 1] - a_rp[a] > a_rp[b + 1] - a_rp[b];
        });
    if (R.sorted_cols)
        std::stable_sort(R.pc.begin(), R.pc.end(), [&](int32_t a, int32_t b) {
            return at_rp[a + 1] - at_rp[a] > at_rp[b + 1] - at_rp[b];
        });
    // panels of A's columns (the table the dual step gathers) and of A^T's
    // columns, i.e. A's rows (the table the primal step gathers)
    R.a_cut = (R.sorted_cols && panels_a > 1) ? deal(R.pc, panels_a)
                                              : even_cuts(n, panels_a);
    R.at_cut = (R.sorted_rows && panels_at > 1) ? deal(R.pr, panels_at)
                                                : even_cuts(m, panels_at);
    std::vector<int32_t> ic((size_t)n), ir((size_t)m);
    for (int64_t j = 0; j < n; ++j) ic[R.pc[j]] = (int32_t)j;
    for (int64_t i = 0; i < m; ++i) ir[R.pr[i]] = (int32_t)i;
    R.a_rp.assign((size_t)m + 1, 0);
    for (int64_t i = 0; i < m; ++i)
        R.a_rp[i + 1] = R.a_rp[i] + (a_rp[R.pr[i] + 1] - a_rp[R.pr[i]]);
    R.a_ci.resize((size_t)nnz);
    R.a_v.resize((size_t)nnz);
    R.apos.resize((size_t)nnz);
    // rows are independent: fill them on a few host threads
    auto fill_rows = [&](int64_t lo, int64_t hi) {
        std::vector<std::pair<int32_t, int32_t>> tmp;
        for (int64_t i2 = lo; i2 < hi; ++i2) {
            const int64_t i = R.pr[i2];
            const int64_t p0 = a_rp[i], L = a_rp[i + 1] - p0;
            tmp.resize((size_t)L);
            for (int64_t q = 0; q < L; ++q)
                tmp[q] = {ic[a_ci[p0 + q]], (int32_t)(p0 + q)};
            std::sort(tmp.begin(), tmp.end());
            const int64_t o = R.a_rp[i2];
            for (int64_t q = 0; q < L; ++q) {
                R.a_ci[o + q] = tmp[q].first;
                R.a_v[o + q] = a_v[tmp[q].second];
                R.apos[o + q] = tmp[q].second;
            }
        }
    };
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(8, nnz / 1000000));
    if (nt == 1) {
        fill_rows(0, m);
    } else {
        std::vector<std::thread> th;
        for (int t = 0; t < nt; ++t)
            th.emplace_back(fill_rows, m * t / nt, m * (t + 1) / nt);
        for (auto &t : th) t.join();
    }
    R.at_rp.assign((size_t)n + 1, 0);
    for (int64_t j = 0; j < n; ++j)
        R.at_rp[j + 1] = R.at_rp[j] + (at_rp[R.pc[j] + 1] - at_rp[R.pc[j]]);
    R.at_ci.resize((size_t)nnz);
    R.at_v.resize((size_t)nnz);
    R.perm.resize((size_t)nnz);
    std::vector<int64_t> cur(R.at_rp.begin(), R.at_rp.end() - 1);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = R.a_rp[i]; p < R.a_rp[i + 1]; ++p) {
            const int64_t q = cur[R.a_ci[p]]++;
            R.at_ci[q] = (int32_t)i;
            R.at_v[q] = R.a_v[p];
            R.perm[p] = (int32_t)q;
        }
    (void)ir;
    return R;
}

// Column panels and XCD affinity.  A random gather is served at a rate that
// falls steeply once its table no longer fits the 4 MB L2 of one XCD.
// Measured on MI355X, random 8-byte gathers per second by table size:
// <= 2 MB 195e9, 4 MB 180e9, 8 MB 110e9, 16 MB 77e9, 32 MB 63e9,
// >= 128 MB 54e9.  The same gathers confined per XCD to 1/P of the table run
// at the rate of the smaller table.  So an SpMV whose table overflows L2 is
// split into P column panels, each handled only by the workgroups that the
// hardware places on the XCDs x with x % P == p (workgroups go to the 8 XCDs
// round-robin by workgroup index).  The price is P stacked rows per row,
// each with its row pointer, its partial sum written and read once, and its
// share of the per-row work of the row-block kernel: measured, about 7 ps
// per stacked row on the whole chip, plus one extra launch that adds the
// partial sums.  Short rows over a table that fits L2 therefore stay whole.
static double gather_rate(double bytes) {
    static const double mb[] = {2, 4, 8, 16, 32, 128};
    static const double g[] = {195e9, 180e9, 110e9, 77e9, 63e9, 54e9};
    const double x = bytes / 1048576.0;
    if (x <= mb[0]) return g[0];
    for (int i = 1; i < 6; ++i)
        if (x <= mb[i]) {
            const double f = std::log(x / mb[i - 1]) / std::log(mb[i] / mb[i - 1]);
            return g[i - 1] * std::pow(g[i] / g[i - 1], f);
        }
    return g[5];
}

int choose_panels(int64_t rows, int64_t cols, int64_t nnz) {
    constexpr double kRow = 7e-12;        // seconds per stacked row
    constexpr double kLaunch = 4e-6;      // the extra launch, seconds
    const double table = 8.0 * (double)cols;
    const double whole = (double)nnz / gather_rate(table);
    double best = 0.95 * whole;           // a split must win clearly
    int bestP = 1;
    for (int P = 2; P <= 8; P *= 2) {
        const double t = (double)nnz / gather_rate(table / P) +
                         kRow * P * (double)rows + kLaunch;
        if (t < best) {
            best = t;
            bestP = P;
        }
    }
    return bestP;
}

// The stacked matrix of P column panels: row p * rows + i holds the entries
// of row i with column in [cut[p], cut[p + 1]) (a contiguous run, since
// columns are sorted within rows); src maps each entry to its position in
// the source arrays.
Panels build_panels(int64_t rows, const int64_t *rp, const int32_t *ci, int P,
                    const std::vector<int64_t> &cut) {
    Panels S;
    const int64_t nnz = rp[rows];
    S.rp.assign((size_t)P * rows + 1, 0);
    std::vector<int64_t> start((size_t)P * rows + 1);
    for (int64_t i = 0; i < rows; ++i) {
        int64_t q = rp[i];
        for (int p = 0; p < P; ++p) {
            start[(size_t)p * rows + i] = q;
            const int64_t e = rp[i + 1];
            int64_t q1 = q;
            while (q1 < e && ci[q1] < cut[p + 1]) ++q1;
            S.rp[(size_t)p * rows + i + 1] = q1 - q;   // length for now
            q = q1;
        }
    }
    S.mask.assign((size_t)rows, 0);
    for (int p = 0; p < P; ++p)
        for (int64_t i = 0; i < rows; ++i)
            if (S.rp[(size_t)p * rows + i + 1] > 0) S.mask[i] |= (uint8_t)(1u << p);
    for (int64_t r = 0; r < (int64_t)P * rows; ++r) S.rp[r + 1] += S.rp[r];
    S.ci.resize((size_t)nnz);
    S.src.resize((size_t)nnz);
    for (int64_t r = 0; r < (int64_t)P * rows; ++r) {
        const int64_t o = S.rp[r], L = S.rp[r + 1] - o, q0 = start[r];
        for (int64_t t = 0; t < L; ++t) {
            S.ci[o + t] = ci[q0 + t];
            S.src[o + t] = (int32_t)(q0 + t);
        }
    }
    return S;
}

// Row blocks of the stacked matrix, built per panel and dealt to the XCDs:
// the blocks of panel p are spread over the XCDs x with x % P == p, and the
// launch order puts XCD x's i-th block at index 8 i + x (empty blocks, r0 ==
// r1, pad queues of unequal length).  Split slots are renumbered to be global.
// No block starts at an empty stacked row, so runs of them (a row whose
// entries all lie in other panels, as in block-structured LPs) cost no
// blocks; the combine reads only the partials of a row's non-empty panels.
HostBins build_panel_blocks(int64_t rows, const int64_t *srp, int P, int tile,
                            int64_t split_threshold, int64_t split_chunk,
                            int max_rows) {
    constexpr int kXcd = 8;
    HostBins out;
    std::vector<std::vector<RowBlock>> q(kXcd);
    for (int p = 0; p < P; ++p) {
        HostBins hb = build_row_blocks(rows, srp + (size_t)p * rows, tile,
                                       split_threshold, split_chunk, max_rows,
                                       true);
        const int32_t roff = (int32_t)((int64_t)p * rows);
        const int slot0 = (int)out.splits.size();
        for (auto sp : hb.splits) {
            sp.row += roff;
            out.splits.push_back(sp);
        }
        out.maxparts = std::max(out.maxparts, hb.maxparts);
        for (int k = 0; k < 3; ++k) out.counts[k] += hb.counts[k];
        const int per = kXcd / P;     // XCDs serving this panel
        for (size_t b = 0; b < hb.blocks.size(); ++b) {
            RowBlock rb = hb.blocks[b];
            rb.r0 += roff;
            rb.r1 += roff;
            if (rb.nparts > 1) rb.slot += slot0;
            q[p + P * (int)(b % per)].push_back(rb);
        }
    }
    size_t depth = 0;
    for (auto &v : q) depth = std::max(depth, v.size());
    out.blocks.reserve(depth * kXcd);
    for (size_t i = 0; i < depth; ++i)
        for (int x = 0; x < kXcd; ++x)
            out.blocks.push_back(i < q[x].size() ? q[x][i]
                                                 : RowBlock{0, 0, 0, 1, -1, 0, 0, 0});
    return out;
}

}  // namespace pdhg
