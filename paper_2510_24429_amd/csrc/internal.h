// internal.h -- declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pdhg.h"

namespace pdhg {

constexpr int kWG = 256;          // threads per workgroup (4 wave64s)
#ifndef PDHG_TILE64
#define PDHG_TILE64 1024
#endif
#ifndef PDHG_TILE32
#define PDHG_TILE32 2048
#endif
constexpr int kTile64 = PDHG_TILE64;  // nonzeros staged per multi-row block, FP64
constexpr int kTile32 = PDHG_TILE32;  // same, FP32 (same LDS bytes)
constexpr int kMaxLevels = 32;
constexpr int kRedBlocks = 512;   // blocks per side of the KKT reduction

// One workgroup's share of a CSR SpMV.  Rows [r0, r1) of one matrix:
//  - several rows (r1 - r0 > 1): their nonzeros (<= tile) are streamed
//    through LDS and summed by groups of lanes per row;
//  - one row (r1 - r0 == 1, nparts == 1): all 256 lanes stride the row and
//    reduce across the workgroup;
//  - one row split over nparts workgroups: part `part` writes a partial sum
//    to slot `slot`; a fix-up pass adds the parts in order.
// A workgroup's rows [r0, r1) and their nonzeros [p0, p1) (the whole row
// for a split row, whose part `part` of `nparts` the workgroup sums into
// partial slot `slot`); r0 == r1 marks an empty padding block.
struct RowBlock {
    int32_t r0, r1, part, nparts, slot, p0, p1, pad;
};

struct SplitRow {
    int32_t row, nparts;
};

struct HostBins {
    std::vector<RowBlock> blocks;
    std::vector<SplitRow> splits;
    int maxparts = 1;
    int64_t counts[3] = {0, 0, 0};   // multi-row, single-row, split parts
};

HostBins build_row_blocks(int64_t rows, const int64_t *rp, int tile,
                          int64_t split_threshold, int64_t split_chunk,
                          int max_rows = 0, bool skip_empty = false);

// Column panels of one SpMV side (see host_csr.cpp): the number of panels P
// (1, 2, 4 or 8) for a matrix of `rows` rows whose gather table has `cols`
// FP64 entries; the stacked panel matrix; its XCD-dealt row blocks.
int choose_panels(int64_t rows, int64_t cols, int64_t nnz);
struct Panels {
    std::vector<int64_t> rp;      // P * rows + 1
    std::vector<int32_t> ci, src;
    std::vector<uint8_t> mask;    // rows: bit p set when stacked row p*rows+i has entries
};
Panels build_panels(int64_t rows, const int64_t *rp, const int32_t *ci, int P,
                    const std::vector<int64_t> &cut);
HostBins build_panel_blocks(int64_t rows, const int64_t *srp, int P, int tile,
                            int64_t split_threshold, int64_t split_chunk,
                            int max_rows = 0);

// The internal (relabeled) problem: row i' of A' is row pr[i'] of A, column
// j' of A' is column pc[j'] of A; apos[p'] is the position in A's arrays of
// A''s nonzero p'; perm[p'] its position in A'^T's arrays.
constexpr double kSkew = 8.0;
struct Relabeled {
    bool sorted_rows = false, sorted_cols = false;
    std::vector<int32_t> pr, pc, apos, perm;
    std::vector<int64_t> a_rp, at_rp;
    std::vector<int32_t> a_ci, at_ci;
    std::vector<double> a_v, at_v;
    std::vector<int64_t> a_cut, at_cut;   // panel boundaries of A' / A'^T columns
};
Relabeled relabel(int64_t m, int64_t n, int64_t nnz, const int64_t *a_rp,
                  const int32_t *a_ci, const double *a_v,
                  const int64_t *at_rp, int panels_a, int panels_at,
                  int sort_rows = -1, int sort_cols = -1);

// Matrix resident on the device: CSR with int32 row pointers.
struct DevCsr {
    int64_t rows = 0, cols = 0, nnz = 0;
    int32_t *rp = nullptr;
    int32_t *ci = nullptr;
    double *v_orig = nullptr;   // loaded values
    double *v64 = nullptr;      // scaled values (D_r A D_c), FP64
    float *v32 = nullptr;       // scaled values rounded to FP32
    // bins for the FP64 tile and the FP32 tile
    RowBlock *blk64 = nullptr;
    int nblk64 = 0;
    RowBlock *blk32 = nullptr;
    int nblk32 = 0;
    SplitRow *split64 = nullptr, *split32 = nullptr;
    int nsplit64 = 0, nsplit32 = 0, maxparts64 = 1, maxparts32 = 1;
    double *part64 = nullptr;   // split partial sums
    float *part32 = nullptr;
    int64_t counts64[3] = {0, 0, 0};
    // column panels (P > 1): the stacked panel matrix (P * rows rows, its
    // values kept equal to v64 / v32 through src), and the partial sums
    int P = 1;
    int stream_nt = 0;          // non-temporal streamed loads (see kernels)
    DevCsr *pan = nullptr;
    int32_t *pan_src = nullptr;
    uint8_t *pan_mask = nullptr;  // per row: which panels hold entries of it
    double *q64 = nullptr;
    float *q32 = nullptr;
};

// Control state of a solve, resident on the device and written only by the
// single-workgroup control kernel (and by the host between solves).
// Per-candidate reduction quantities.  Q_FX2 / Q_FY2 are sums of squares of
// the difference between the two candidates (||x - T_x(z)||^2 etc. for the
// Halpern variant), accumulated under candidate 1.
enum { Q_RP2, Q_RPMAX, Q_SRP2, Q_BY, Q_DY2, Q_RD2, Q_RDMAX, Q_SRD2, Q_CX,
       Q_LZ, Q_DX2, Q_FX2, Q_FY2, Q_NQ };
enum { S_RELP, S_RELD, S_RELG, S_MAXR, S_POBJ, S_DOBJ, S_NRP, S_NRD,
       S_RPINF, S_RDINF, S_SP2, S_SD2, S_SG, S_DX2, S_DY2, S_FIN, S_NS };

struct State {
    double tau, sigma, omega, eta;
    double K_last, K_prev;
    double nb, nc;                  // ||b||_2, ||c||_2 of the unscaled data
    double eps_rel, beta_suff, beta_nec, beta_art, omega_theta;
    double reflect;                 // Halpern reflection
    double pid_kp, pid_ki, pid_kd;  // PID gains of the primal weight
    double pid_int, pid_eprev;      // its integral and last error
    int omega_rule;                 // 0 smoothed, 1 PID
    int stop_on;                    // stop measure: 0 maxresid, 1 rel_p, 2 rel_d
    int polish;                     // feasibility polishing enabled
    int polish_due;                 // this evaluation asks for an attempt
    int polish_cand;                // from candidate 0 or 1
    int pad_polish;
    long long next_polish;          // earliest iteration of the next attempt
    double fx2, fy2;                // ||z - T(z)||^2 parts at the last evaluation
    long long k;                    // iterations done
    long long t_base;               // iterations since the last restart
    int status;
    int copy_pending;               // 1: restart / final copy to apply
    int copy_avg;                   // candidate copied into the current iterate
    int set_last;                   // 1: restart point <- current afterwards
    int restarts;
    int next_level, n_levels, literal;
    int snap_count;
    int snap_first, snap_n, snap_cand;
    int returned_cand;
    int n_log, log_cap;
    int last_ncand;
    int variant;                    // 0 averaged, 1 reflected Halpern
    double levels[kMaxLevels];
    double stats[2][S_NS];
    double snap_level[kMaxLevels];
    long long snap_iter[kMaxLevels];
    double snap_mr[kMaxLevels];
    int snap_cand_of[kMaxLevels];
};

// Vectors of one precision for the bulk iteration.
template <typename T>
struct Iter {
    T *x = nullptr, *y = nullptr, *xbar = nullptr, *ybar = nullptr;
    T *xl = nullptr, *yl = nullptr;       // last restart point
    T *ax = nullptr;                      // A~ x of the current iterate
    T *ax0 = nullptr;                     // A~ x of the Halpern anchor
    T *cs = nullptr, *bs = nullptr, *ls = nullptr;   // scaled data in T
};

// ---- launchers (kernels.hip) -------------------------------------------

// out = M in  (M = A~ / A / A~32 chosen by the caller through `vals`)
void spmv_f64(const DevCsr &M, const double *vals, const double *in,
              double *out, hipStream_t s);
void spmv_f64_in32(const DevCsr &M, const double *vals, const float *in,
                   double *out, hipStream_t s);
void spmv_f32(const DevCsr &M, const float *in, float *out, hipStream_t s);

template <typename T>
void launch_primal(const DevCsr &At, const Iter<T> &v, bool has_l,
                   bool avg, const State *st, int off, hipStream_t s);
template <typename T>
void launch_dual(const DevCsr &A, const Iter<T> &v, bool avg,
                 const State *st, int off, hipStream_t s);
// Halpern iteration: primal writes x^ = T_x(z) into v.xbar and the combined
// x; dual gathers v.xbar and combines y and A~x with the anchors (xl, yl,
// ax0).
template <typename T>
void launch_primal_halpern(const DevCsr &At, const Iter<T> &v, bool has_l,
                           const State *st, int off, hipStream_t s);
template <typename T>
void launch_dual_halpern(const DevCsr &A, const Iter<T> &v, const State *st,
                         int off, hipStream_t s);
// Halpern evaluation: T(z) of the current iterate in FP64 arithmetic, into
// v.xbar / v.ybar, with aty = A~^T y and axh = A~ x^ (FP64); axc is A~ x of
// the current iterate (FP64).
template <typename T>
void launch_eval_T(const DevCsr &A, const DevCsr &At, const Iter<T> &v,
                   bool has_l, const double *cs, const double *bs,
                   const double *ls, const State *st, double *aty,
                   double *axh, const double *axc, hipStream_t s);

void launch_kkt_reduce(int ncand, const void *x0, const void *y0,
                       const void *x1, const void *y1, bool f32,
                       const double *ax0, const double *aty0,
                       const double *ax1, const double *aty1,
                       const void *xl, const void *yl, const double *bs,
                       const double *cs, const double *ls, const double *dr,
                       const double *dc, int64_t m, int64_t n,
                       double *partial, hipStream_t s);
void launch_control(State *st, const double *partial, int ncand, int batch,
                    int initial, double *log, hipStream_t s);
// When the evaluation asked for a polishing attempt: the candidate it chose,
// unscaled (D_c x, D_r y) in FP64, into xs / ys (before any restart moves it).
void launch_polish_stash(const State *st, bool f32, const void *x0,
                         const void *y0, const void *x1, const void *y1,
                         const double *dr, const double *dc, double *xs,
                         double *ys, int64_t m, int64_t n, hipStream_t s);
void launch_advance(State *st, int batch, hipStream_t s);
void launch_set_status(State *st, int status, hipStream_t s);
void launch_restart_apply(State *st, bool f32, void *x, void *y, void *ax,
                          void *xbar, void *ybar, const double *ax_avg,
                          void *xl, void *yl, void *ax0, int64_t m, int64_t n,
                          hipStream_t s);
void launch_snapshot_pack(const State *st, bool f32, const void *x0,
                          const void *y0, const void *x1, const void *y1,
                          const double *aty0, const double *aty1,
                          const double *cs, const double *dr, const double *dc,
                          const int32_t *pr, const int32_t *pc, double *slots,
                          int64_t m, int64_t n, hipStream_t s);

// Ruiz: rho_r = max over row r of M of |(D_r,i a_ij) D_c,j| for the entry's
// (i, j) in A.  d_row scales M's rows and d_col its columns; transposed = 1
// when M is A^T (the first factor is then d_col).  The update divides d by
// sqrt(rho) (a zero maximum counts as 1).
void launch_ruiz_rowmax(const DevCsr &M, const double *d_row,
                        const double *d_col, int transposed, double *rho,
                        hipStream_t s);
void launch_ruiz_update(double *d, const double *rho, int64_t k,
                        hipStream_t s);
// Entries of the rows of A scaled by fixed factors:
// out[p] = (rs[row] * v[p]) * cs[col]; out32 (optional) gets the FP32 copy.
void launch_scale_values(const DevCsr &M, const double *v, const double *rs,
                         const double *cs, double *out, float *out32,
                         hipStream_t s);

// Deterministic FP64 reductions: partial sums of squares / dot products by
// blocks, then a fixed-order finish in one workgroup.
void launch_dot(const double *a, const double *b, int64_t k, double *partial,
                double *result, hipStream_t s);
void launch_scale_vec(double *dst, const double *src, const double *factor,
                      int64_t k, int mode, hipStream_t s);
void launch_fill(double *p, double v, int64_t k, hipStream_t s);
void launch_fill32(float *p, float v, int64_t k, hipStream_t s);
void launch_to_f32(float *dst, const double *src, int64_t k, hipStream_t s);
void launch_to_f64(double *dst, const float *src, int64_t k, hipStream_t s);
// elementwise: out = a * b (mode 0), a / b (mode 1), a * b with b a scalar
// pointer (mode 2)
void launch_ew(double *out, const double *a, const double *b, int64_t k,
               int mode, hipStream_t s);
// Unscaled x = D_c xs, y = D_r ys, z = max(0, (cs - aty) / D_c), each
// written at its original index (x[pc[j]], y[pr[i]], z[pc[j]]).
void launch_unscale_xyz(const double *xs, const double *ys,
                        const double *aty, const double *cs, const double *dr,
                        const double *dc, const int32_t *pr, const int32_t *pc,
                        double *x, double *y, double *z, int64_t m, int64_t n,
                        hipStream_t s);
void launch_unscale_xyz32(const float *xs, const float *ys,
                          const double *aty, const double *cs,
                          const double *dr, const double *dc,
                          const int32_t *pr, const int32_t *pc, double *x,
                          double *y, double *z, int64_t m, int64_t n,
                          hipStream_t s);
// dst[idx[i]] = src[i] (scatter) / dst[i] = src[idx[i]] (gather)
void launch_permute(double *dst, const double *src, const int32_t *perm,
                    int64_t k, hipStream_t s);
void launch_gather(double *dst, const double *src, const int32_t *idx,
                   int64_t k, hipStream_t s);

// Refinement (FP64): residual data of the correction LP and its update.
void launch_refine_rhs(const double *bs, const double *ax, const double *cs,
                       const double *aty, const double *xs, const double *ls,
                       double DP, double DD, double *bh, double *ch,
                       double *lh, int64_t m, int64_t n, hipStream_t s);
void launch_refine_delta(const double *bs, const double *ax, const double *cs,
                         const double *aty, const double *xs,
                         const double *ls, const double *dr, const double *dc,
                         int64_t m, int64_t n, double *partial, double *out2,
                         hipStream_t s);
// x <- max(l, x + xh / DP), y <- y + yh / DD (ls may be NULL: l = 0)
template <typename T>
void launch_refine_update(double *xs, double *ys, const T *xh, const T *yh,
                          const double *ls, double DP, double DD, int64_t m,
                          int64_t n, hipStream_t s);
void launch_norm_unscaled(const double *vs, const double *d, int64_t k,
                          double *partial, double *result, hipStream_t s);

// Adjoint kernels (template over T = float/double).
template <typename T>
void launch_adj_dual_bwd(const DevCsr &At, const T *gy, const T *gx_in,
                         const T *x1, const T *ls, bool has_l, T *gx_out,
                         T *gv, T *gc, double tau, double sigma,
                         hipStream_t s);
template <typename T>
void launch_adj_primal_bwd(const DevCsr &A, const T *gv, const T *gy_in,
                           T *gy_out, T *gb, double tau, double sigma,
                           hipStream_t s);
template <typename T>
void launch_adj_gA(const DevCsr &A, const int32_t *rowidx, const T *y0,
                   const T *gy1, const T *gv, const T *x0, const T *x1,
                   T *gA, double tau, double sigma, hipStream_t s);

// Gather-rate probe: indices of n streamed pairs, chunk per workgroup, each
// workgroup confined to its panel of a table of `table` entries; the probe
// kernel streams the pairs and sums val * table[idx] per workgroup into out.
void launch_probe_fill(int32_t *idx, int64_t n, int64_t chunk, int64_t table,
                       int P, uint64_t seed, hipStream_t s);
template <typename T>
void launch_gather_probe(const int32_t *idx, const T *val, const T *table,
                         int64_t chunk, int64_t n, bool nt, T *out,
                         hipStream_t s);

}  // namespace pdhg
