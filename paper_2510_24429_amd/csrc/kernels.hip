// kernels.hip -- HIP kernels for gfx950 (CDNA4, wave64).
//
// All sparse products go through one row-block kernel: each workgroup takes
// a descriptor (a run of short rows, one long row, or one part of a split
// row) built on the host from the row lengths.  Multi-row blocks stream
// their nonzeros, fully coalesced, into LDS and sum each row with a group of
// lanes sized to the block's row count; single long rows are strided by the
// whole workgroup and reduced across its four waves.  The PDHG updates are
// epilogues of these products, so every iteration is two kernels.  No
// atomics: every sum has a fixed order for a given matrix, so repeated runs
// are bitwise identical.
#include <cmath>

#include <type_traits>

#include "control.h"
#include "internal.h"

namespace pdhg {

namespace {

constexpr int kFixThreads = 64;

// Loads of the streamed CSR arrays (indices and values, each read once per
// SpMV), plain or non-temporal.  Measured on MI355X: plain loads are faster
// while the gathered table fits comfortably in L2 (9.4M streamed pairs with
// one random gather each from a 1.6 MB table: 45.5 us plain, 54.6 us
// non-temporal; the power-law steps 7,120 -> 7,773 iterations/s), while
// non-temporal loads keep a 5 MB gather panel in L2 (multicommodity, FP32:
// 3,828 plain, 4,294 non-temporal).  Each matrix side picks one at load.
template <bool NT, typename T>
__device__ __forceinline__ T sload(const T *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Four consecutive streamed entries starting at a multiple of 4, as 16-byte
// loads (index arrays and value arrays are padded to a multiple of 4).
template <bool NT>
__device__ __forceinline__ void ld4(const int32_t *p, int (&o)[4]) {
    const v4i v = sload<NT>((const v4i *)p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <bool NT>
__device__ __forceinline__ void ld4(const double *p, double (&o)[4]) {
    const v2d a = sload<NT>((const v2d *)p);
    const v2d b = sload<NT>((const v2d *)(p + 2));
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
template <bool NT>
__device__ __forceinline__ void ld4(const float *p, float (&o)[4]) {
    const v4f v = sload<NT>((const v4f *)p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Sum over the 256 threads of a workgroup; every thread gets the result.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *sred) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sred[w] = v;
    __syncthreads();
    return (sred[0] + sred[1]) + (sred[2] + sred[3]);
}

__device__ __forceinline__ double block_max(double v, double *sred) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sred[w] = v;
    __syncthreads();
    return fmax(fmax(sred[0], sred[1]), fmax(sred[2], sred[3]));
}

// ---------------------------------------------------------------- elements

// One nonzero's contribution v[p] * x[ci[p]].  fetch4() reads four streamed
// indices and values, apply() gathers x and multiplies; splitting the two
// lets a thread issue all of its index/value loads, then all of its gathers,
// before waiting on any of them.
// (The load kind is a template parameter: a runtime branch between the two
// kinds of otherwise identical loads was merged by the compiler into plain
// loads.)
template <typename MT, typename VT, typename Acc, bool NT>
struct SpmvElem {
    const int32_t *ci;
    const MT *v;
    const VT *x;
    // entries base..base+3 (base a multiple of 4)
    __device__ __forceinline__ void fetch4(int base, int (&j)[4],
                                           MT (&a)[4]) const {
        ld4<NT>(ci + base, j);
        ld4<NT>(v + base, a);
    }
    __device__ __forceinline__ Acc apply(int j, MT a) const {
        return (Acc)a * (Acc)x[j];
    }
};

// ---------------------------------------------------------------- epilogues

// An epilogue may split into pre(r), the loads of its own operands of row r,
// and fin(r, s, pre), the update with the row sum s; multi-row blocks then
// issue the loads at their start, ahead of the row sums (operator() is
// fin(r, s, pre(r))).  Epilogues without a Pre type run after the sums.
template <class Epi, class = void>
struct has_pre : std::false_type {};
template <class Epi>
struct has_pre<Epi, std::void_t<typename Epi::Pre>> : std::true_type {};
struct NoPre {};
template <class Epi, bool = has_pre<Epi>::value>
struct PreOf {
    using type = NoPre;
};
template <class Epi>
struct PreOf<Epi, true> {
    using type = typename Epi::Pre;
};

template <typename OutT, typename Acc>
struct StoreEpi {
    OutT *out;
    __device__ __forceinline__ bool begin() { return true; }
    __device__ __forceinline__ void operator()(int r, Acc s) const {
        out[r] = (OutT)s;
    }
};

// Panel pass: row r of the stacked panel matrix stores its partial sum; the
// wrapped epilogue's begin() still decides whether the pass runs at all.
template <class Epi, typename Acc>
struct PanelEpi {
    Epi e;
    Acc *q;
    __device__ __forceinline__ bool begin() { return e.begin(); }
    __device__ __forceinline__ void operator()(int r, Acc s) const { q[r] = s; }
};

// Fused primal step over a row j of A~^T:
//   x_j <- max(l_j, x_j - tau (c_j - g_j)),  xbar_j <- xbar_j + (x_j - xbar_j)/t
template <typename T, bool HAS_L, bool AVG>
struct PrimalEpi {
    T *x, *xbar;
    const T *c, *l;
    const State *st;
    int off;
    T tau;
    T t;
    __device__ __forceinline__ bool begin() {
        if (st->status != PDHG_RUNNING) return false;
        tau = (T)st->tau;
        t = (T)(double)(st->t_base + off + 1);
        return true;
    }
    struct Pre {
        T x, c, l, xb;
    };
    __device__ __forceinline__ Pre pre(int j) const {
        return {x[j], c[j], HAS_L ? l[j] : (T)0, AVG ? xbar[j] : (T)0};
    }
    __device__ __forceinline__ void fin(int j, T g, const Pre &p) const {
        const T v = p.x - tau * (p.c - g);
        const T xn = v < p.l ? p.l : v;
        x[j] = xn;
        if (AVG) xbar[j] = p.xb + (xn - p.xb) / t;
    }
    __device__ __forceinline__ void operator()(int j, T g) const { fin(j, g, pre(j)); }
};

// Fused extrapolated dual step over a row i of A~ (q = (A~ x_new)_i):
//   y_i <- y_i + sigma (b_i - (2 q - (A~ x_old)_i)),  (A~ x)_i <- q,  ybar
template <typename T, bool AVG>
struct DualEpi {
    T *y, *ybar, *ax;
    const T *b;
    const State *st;
    int off;
    T sigma;
    T t;
    __device__ __forceinline__ bool begin() {
        if (st->status != PDHG_RUNNING) return false;
        sigma = (T)st->sigma;
        t = (T)(double)(st->t_base + off + 1);
        return true;
    }
    struct Pre {
        T y, b, a, yb;
    };
    __device__ __forceinline__ Pre pre(int i) const {
        return {y[i], b[i], ax[i], AVG ? ybar[i] : (T)0};
    }
    __device__ __forceinline__ void fin(int i, T q, const Pre &p) const {
        const T yn = p.y + sigma * (p.b - ((q + q) - p.a));
        y[i] = yn;
        ax[i] = q;
        if (AVG) ybar[i] = p.yb + (yn - p.yb) / t;
    }
    __device__ __forceinline__ void operator()(int i, T q) const { fin(i, q, pre(i)); }
};

// Reflected Halpern step, primal part over a row j of A~^T:
//   x^_j = max(l_j, x_j - tau (c_j - g_j))   (kept for the dual part)
//   x_j <- lambda ((1 + rho) x^_j - rho x_j) + (1 - lambda) x0_j
// with lambda = t / (t + 1) for the t-th step since the anchor x0.
template <typename T, bool HAS_L>
struct PrimalHalpernEpi {
    T *x, *xh;
    const T *c, *l, *x0;
    const State *st;
    int off;
    T tau, lam, rho;
    __device__ __forceinline__ bool begin() {
        if (st->status != PDHG_RUNNING) return false;
        tau = (T)st->tau;
        const double t = (double)(st->t_base + off + 1);
        lam = (T)(t / (t + 1.0));
        rho = (T)st->reflect;
        return true;
    }
    struct Pre {
        T x, c, l, x0;
    };
    __device__ __forceinline__ Pre pre(int j) const {
        return {x[j], c[j], HAS_L ? l[j] : (T)0, x0[j]};
    }
    __device__ __forceinline__ void fin(int j, T g, const Pre &p) const {
        const T v = p.x - tau * (p.c - g);
        const T xhv = v < p.l ? p.l : v;
        xh[j] = xhv;
        x[j] = lam * (((T)1 + rho) * xhv - rho * p.x) + ((T)1 - lam) * p.x0;
    }
    __device__ __forceinline__ void operator()(int j, T g) const { fin(j, g, pre(j)); }
};

// Reflected Halpern step, dual part over a row i of A~ (q = (A~ x^)_i):
//   y^_i = y_i + sigma (b_i - (2 q - (A~x)_i))
//   y_i  <- lambda ((1 + rho) y^_i - rho y_i) + (1 - lambda) y0_i
//   (A~x)_i <- lambda ((1 + rho) q - rho (A~x)_i) + (1 - lambda) (A~x0)_i
template <typename T>
struct DualHalpernEpi {
    T *y, *ax;
    const T *b, *y0, *ax0;
    const State *st;
    int off;
    T sigma, lam, rho;
    __device__ __forceinline__ bool begin() {
        if (st->status != PDHG_RUNNING) return false;
        sigma = (T)st->sigma;
        const double t = (double)(st->t_base + off + 1);
        lam = (T)(t / (t + 1.0));
        rho = (T)st->reflect;
        return true;
    }
    struct Pre {
        T a, y, b, y0, a0;
    };
    __device__ __forceinline__ Pre pre(int i) const {
        return {ax[i], y[i], b[i], y0[i], ax0[i]};
    }
    __device__ __forceinline__ void fin(int i, T q, const Pre &p) const {
        const T yhv = p.y + sigma * (p.b - ((q + q) - p.a));
        y[i] = lam * (((T)1 + rho) * yhv - rho * p.y) + ((T)1 - lam) * p.y0;
        ax[i] = lam * (((T)1 + rho) * q - rho * p.a) + ((T)1 - lam) * p.a0;
    }
    __device__ __forceinline__ void operator()(int i, T q) const { fin(i, q, pre(i)); }
};

// Evaluation of T(z) in FP64 arithmetic (storage T): primal part over a row j
// of A~^T records A~^T y and x^ = max(l, x - tau (c - A~^T y)).
template <typename T, bool HAS_L>
struct PrimalEvalEpi {
    const T *x;
    const double *c, *l;
    T *xh;
    double *aty;
    const State *st;
    double tau;
    __device__ __forceinline__ bool begin() {
        tau = st->tau;
        return true;
    }
    __device__ __forceinline__ void operator()(int j, double g) const {
        aty[j] = g;
        const double v = (double)x[j] - tau * (c[j] - g);
        const double lj = HAS_L ? l[j] : 0.0;
        xh[j] = (T)(v < lj ? lj : v);
    }
};

// ... dual part over a row i of A~ (q = (A~ x^)_i) records A~ x^ and
// y^ = y + sigma (b - (2 q - A~x)).
template <typename T>
struct DualEvalEpi {
    const T *y;
    const double *axc, *b;
    T *yh;
    double *axh;
    const State *st;
    double sigma;
    __device__ __forceinline__ bool begin() {
        sigma = st->sigma;
        return true;
    }
    __device__ __forceinline__ void operator()(int i, double q) const {
        axh[i] = q;
        yh[i] = (T)((double)y[i] + sigma * (b[i] - ((q + q) - axc[i])));
    }
};

// Adjoint of the dual step, over a row j of A~^T (s = (A~^T gy_{k+1})_j):
//   gxbar = -sigma s;  g = gx_{k+1} + 2 gxbar;  gv = 1[x_{k+1} > l] g
//   gx_k = gv - gxbar;  gc -= tau gv
template <typename T, bool HAS_L>
struct AdjDualEpi {
    const T *gx_in, *x1, *l;
    T *gx_out, *gv, *gc;
    T tau, sigma;
    __device__ __forceinline__ bool begin() { return true; }
    __device__ __forceinline__ void operator()(int j, T s) const {
        const T gxbar = -sigma * s;
        const T g = gx_in[j] + (gxbar + gxbar);
        const T lj = HAS_L ? l[j] : (T)0;
        const T v = x1[j] > lj ? g : (T)0;
        gv[j] = v;
        gx_out[j] = v - gxbar;
        gc[j] = gc[j] - tau * v;
    }
};

// Adjoint of the primal step, over a row i of A~ (s = (A~ gv)_i):
//   gy_k = gy_{k+1} + tau s;  gb += sigma gy_{k+1}
template <typename T>
struct AdjPrimalEpi {
    const T *gy_in;
    T *gy_out, *gb;
    T tau, sigma;
    __device__ __forceinline__ bool begin() { return true; }
    __device__ __forceinline__ void operator()(int i, T s) const {
        const T g = gy_in[i];
        gy_out[i] = g + tau * s;
        gb[i] = gb[i] + sigma * g;
    }
};

// ---------------------------------------------------------------- kernels

template <typename Acc, int TILE, class Elem, class Epi>
__global__ __launch_bounds__(kWG) void k_rowblock(
    const RowBlock *__restrict__ blks, const int32_t *__restrict__ rp,
    Elem elem, Epi epi_in, Acc *__restrict__ part, int maxparts) {
    constexpr int U = TILE / kWG;     // nonzeros per thread in a full tile
    using MT = decltype(elem.v[0] + 0);
    __shared__ Acc s_prod[TILE];
    __shared__ Acc s_sum[kWG];
    __shared__ int s_rp[TILE + 1];
    __shared__ Acc s_red[4];
    Epi epi = epi_in;
    if (!epi.begin()) return;
    const RowBlock b = blks[blockIdx.x];
    if (b.r1 == b.r0) return;         // padding of an XCD queue
    const int tid = threadIdx.x;
    if (b.r1 - b.r0 == 1) {
        // one row: the workgroup strides it in aligned groups of four
        // nonzeros per lane (16-byte index and value loads), two groups in
        // flight; entries outside [p0, p1) are masked and never gathered
        int p0 = b.p0, p1 = b.p1;
        if (b.nparts > 1) {
            const int chunk = (p1 - p0 + b.nparts - 1) / b.nparts;
            p0 = p0 + b.part * chunk;
            p1 = min(p1, p0 + chunk);
        }
        Acc s0 = (Acc)0, s1 = (Acc)0;
        int base = (p0 & ~3) + 4 * tid;
        for (; base + 4 * kWG < p1; base += 8 * kWG) {
            int j0[4], j1[4];
            MT a0[4], a1[4];
            elem.fetch4(base, j0, a0);
            elem.fetch4(base + 4 * kWG, j1, a1);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int p = base + u;
                if (p >= p0) s0 += elem.apply(j0[u], a0[u]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int p = base + 4 * kWG + u;
                if (p < p1) s1 += elem.apply(j1[u], a1[u]);
            }
        }
        if (base < p1) {
            int j0[4];
            MT a0[4];
            elem.fetch4(base, j0, a0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int p = base + u;
                if (p >= p0 && p < p1) s0 += elem.apply(j0[u], a0[u]);
            }
        }
        Acc s = block_sum(s0 + s1, s_red);
        if (tid == 0) {
            if (b.nparts > 1)
                part[b.slot * maxparts + b.part] = s;
            else
                epi(b.r0, s);
        }
        return;
    }
    // several rows: stage their row pointers in LDS, stream their nonzeros
    // (contiguous, <= TILE - 3) into LDS in aligned groups of four per lane
    // (16-byte loads), index and value loads first, then the gathers
    const int R = b.r1 - b.r0;
    // the epilogue's own operands of this thread's row, loaded first
    typename PreOf<Epi>::type pre{};
    if constexpr (has_pre<Epi>::value)
        if (R <= kWG && tid < R) pre = epi.pre(b.r0 + tid);
    const int p0 = b.p0;
    const int nz = b.p1 - p0;
    for (int r = tid; r <= R; r += kWG) s_rp[r] = rp[b.r0 + r] - p0;
    {
        const int a0 = p0 & ~3;
        constexpr int G4 = U / 4;      // groups of four per lane
        int jj[G4][4];
        MT aa[G4][4];
#pragma unroll
        for (int g = 0; g < G4; ++g) {
            const int base = a0 + 4 * (tid + g * kWG);
            if (base < p0 + nz) elem.fetch4(base, jj[g], aa[g]);
        }
#pragma unroll
        for (int g = 0; g < G4; ++g) {
            const int base = a0 + 4 * (tid + g * kWG);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = base + u - p0;
                if (q >= 0 && q < nz) s_prod[q] = elem.apply(jj[g][u], aa[g][u]);
            }
        }
    }
    __syncthreads();
    if (R <= kWG) {
        // a power-of-two group of lanes per row sums it from LDS
        int G = 64;
        while (G * R > kWG) G >>= 1;
        const int r = tid / G, lane = tid & (G - 1);
        Acc s = (Acc)0;
        if (r < R) {
            const int q1 = s_rp[r + 1];
            for (int q = s_rp[r] + lane; q < q1; q += G) s += s_prod[q];
        }
        for (int o = G >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (r < R && lane == 0) s_sum[r] = s;
        __syncthreads();
        // epilogue on consecutive rows by consecutive threads
        if (tid < R) {
            if constexpr (has_pre<Epi>::value)
                epi.fin(b.r0 + tid, s_sum[tid], pre);
            else
                epi(b.r0 + tid, s_sum[tid]);
        }
    } else {
        for (int r = tid; r < R; r += kWG) {
            const int q1 = s_rp[r + 1];
            Acc s = (Acc)0;
            for (int q = s_rp[r]; q < q1; ++q) s += s_prod[q];
            epi(b.r0 + r, s);
        }
    }
}

// Finish split rows: add the parts in order, then the epilogue.
template <typename Acc, class Epi>
__global__ __launch_bounds__(kFixThreads) void k_split_fix(
    const SplitRow *__restrict__ sp, int nsplit, const Acc *__restrict__ part,
    int maxparts, Epi epi_in) {
    Epi epi = epi_in;
    if (!epi.begin()) return;
    const int t = blockIdx.x * kFixThreads + threadIdx.x;
    if (t >= nsplit) return;
    Acc s = (Acc)0;
    const SplitRow r = sp[t];
    for (int q = 0; q < r.nparts; ++q) s += part[t * maxparts + q];
    epi(r.row, s);
}

// Rows of a panelled matrix: the partial sums of row i (stacked rows
// p * rows + i) over the panels that hold entries of it (bits of mask[i];
// all panels when mask is null), added in panel order, then the epilogue.
// Partials of empty stacked rows are neither written nor read; skipping
// them drops only exact zeros.
template <typename Acc, class Epi>
__global__ __launch_bounds__(kWG) void k_panel_combine(
    const Acc *__restrict__ q, const uint8_t *__restrict__ mask, int P,
    int rows, Epi epi_in) {
    Epi epi = epi_in;
    if (!epi.begin()) return;
    for (int i = blockIdx.x * kWG + threadIdx.x; i < rows; i += gridDim.x * kWG) {
        const unsigned m = mask ? mask[i] : 0xffu;
        Acc s = (Acc)0;
        for (int p = 0; p < P; ++p)
            if (m & (1u << p)) s += q[(int64_t)p * rows + i];
        epi(i, s);
    }
}

template <typename Acc, int TILE, class Elem, class Epi>
void run_rowblock(const RowBlock *blk, int nblk, const SplitRow *split,
                  int nsplit, Acc *part, int maxparts, const int32_t *rp,
                  Elem elem, Epi epi, hipStream_t s) {
    if (nblk > 0)
        hipLaunchKernelGGL((k_rowblock<Acc, TILE, Elem, Epi>), dim3(nblk),
                           dim3(kWG), 0, s, blk, rp, elem, epi, part,
                           maxparts);
    if (nsplit > 0)
        hipLaunchKernelGGL((k_split_fix<Acc, Epi>),
                           dim3((nsplit + kFixThreads - 1) / kFixThreads),
                           dim3(kFixThreads), 0, s, split, nsplit, part,
                           maxparts, epi);
}

int grid_for(int64_t k, int per = kWG, int cap = 8192) {
    int64_t g = (k + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// FP64 accumulation always uses the FP64 bins; FP32 accumulation the FP32
// bins (twice the nonzeros per tile for the same LDS bytes).
template <typename Acc, class Elem, class Epi>
void run_bins(const DevCsr &M, Elem e, Epi p, hipStream_t s) {
    if constexpr (std::is_same<Acc, double>::value)
        run_rowblock<double, kTile64>(M.blk64, M.nblk64, M.split64, M.nsplit64,
                                      M.part64, M.maxparts64, M.rp, e, p, s);
    else
        run_rowblock<float, kTile32>(M.blk32, M.nblk32, M.split32, M.nsplit32,
                                     M.part32, M.maxparts32, M.rp, e, p, s);
}

// out-row r of M x epilogue, with M's values `vals` (its scaled FP64 or FP32
// values, or others).  A panelled M runs its scaled values through the panel
// twin (XCD-dealt panel pass, then the combine with the epilogue); any other
// value array takes the plain bins.
template <typename Acc, typename MT, typename VT, class Epi>
void rb_spmv(const DevCsr &M, const MT *vals, const VT *in, Epi e,
             hipStream_t s) {
    const MT *tv = nullptr;
    if (M.pan) {
        if constexpr (std::is_same<MT, double>::value) {
            if (vals == M.v64) tv = M.pan->v64;
        } else {
            if (vals == M.v32) tv = M.pan->v32;
        }
    }
    if (!tv) {
        if (M.stream_nt)
            run_bins<Acc>(M, SpmvElem<MT, VT, Acc, true>{M.ci, vals, in}, e, s);
        else
            run_bins<Acc>(M, SpmvElem<MT, VT, Acc, false>{M.ci, vals, in}, e, s);
        return;
    }
    Acc *q;
    if constexpr (std::is_same<Acc, double>::value)
        q = M.q64;
    else
        q = M.q32;
    if (M.stream_nt)
        run_bins<Acc>(*M.pan, SpmvElem<MT, VT, Acc, true>{M.pan->ci, tv, in},
                      PanelEpi<Epi, Acc>{e, q}, s);
    else
        run_bins<Acc>(*M.pan, SpmvElem<MT, VT, Acc, false>{M.pan->ci, tv, in},
                      PanelEpi<Epi, Acc>{e, q}, s);
    hipLaunchKernelGGL((k_panel_combine<Acc, Epi>),
                       dim3(grid_for(M.rows, kWG, 4096)), dim3(kWG), 0, s, q,
                       M.pan_mask, M.P, (int)M.rows, e);
}

}  // namespace

// ======================================================================= SpMV

void spmv_f64(const DevCsr &M, const double *vals, const double *in,
              double *out, hipStream_t s) {
    rb_spmv<double>(M, vals, in, StoreEpi<double, double>{out}, s);
}

void spmv_f64_in32(const DevCsr &M, const double *vals, const float *in,
                   double *out, hipStream_t s) {
    rb_spmv<double>(M, vals, in, StoreEpi<double, double>{out}, s);
}

void spmv_f32(const DevCsr &M, const float *in, float *out, hipStream_t s) {
    rb_spmv<float>(M, (const float *)M.v32, in, StoreEpi<float, float>{out}, s);
}

// ============================================================ PDHG iteration

template <typename T, class Epi>
static void rbT(const DevCsr &M, const T *in, Epi e, hipStream_t s) {
    if constexpr (sizeof(T) == 8)
        rb_spmv<double>(M, (const double *)M.v64, in, e, s);
    else
        rb_spmv<float>(M, (const float *)M.v32, in, e, s);
}

template <typename T>
void launch_primal(const DevCsr &At, const Iter<T> &v, bool has_l, bool avg,
                   const State *st, int off, hipStream_t s) {
    if (has_l) {
        if (avg)
            rbT<T>(At, v.y, PrimalEpi<T, true, true>{v.x, v.xbar, v.cs, v.ls, st, off}, s);
        else
            rbT<T>(At, v.y, PrimalEpi<T, true, false>{v.x, v.xbar, v.cs, v.ls, st, off}, s);
    } else {
        if (avg)
            rbT<T>(At, v.y, PrimalEpi<T, false, true>{v.x, v.xbar, v.cs, v.ls, st, off}, s);
        else
            rbT<T>(At, v.y, PrimalEpi<T, false, false>{v.x, v.xbar, v.cs, v.ls, st, off}, s);
    }
}

template <typename T>
void launch_dual(const DevCsr &A, const Iter<T> &v, bool avg, const State *st,
                 int off, hipStream_t s) {
    if (avg)
        rbT<T>(A, v.x, DualEpi<T, true>{v.y, v.ybar, v.ax, v.bs, st, off}, s);
    else
        rbT<T>(A, v.x, DualEpi<T, false>{v.y, v.ybar, v.ax, v.bs, st, off}, s);
}

template <typename T>
void launch_primal_halpern(const DevCsr &At, const Iter<T> &v, bool has_l,
                           const State *st, int off, hipStream_t s) {
    if (has_l)
        rbT<T>(At, v.y, PrimalHalpernEpi<T, true>{v.x, v.xbar, v.cs, v.ls, v.xl, st, off}, s);
    else
        rbT<T>(At, v.y, PrimalHalpernEpi<T, false>{v.x, v.xbar, v.cs, v.ls, v.xl, st, off}, s);
}

template <typename T>
void launch_dual_halpern(const DevCsr &A, const Iter<T> &v, const State *st,
                         int off, hipStream_t s) {
    rbT<T>(A, (const T *)v.xbar, DualHalpernEpi<T>{v.y, v.ax, v.bs, v.yl, v.ax0, st, off}, s);
}

template <typename T>
void launch_eval_T(const DevCsr &A, const DevCsr &At, const Iter<T> &v,
                   bool has_l, const double *cs, const double *bs,
                   const double *ls, const State *st, double *aty,
                   double *axh, const double *axc, hipStream_t s) {
    const double *atv = At.v64, *av = A.v64;
    if (has_l)
        rb_spmv<double>(At, atv, (const T *)v.y,
                        PrimalEvalEpi<T, true>{v.x, cs, ls, v.xbar, aty, st}, s);
    else
        rb_spmv<double>(At, atv, (const T *)v.y,
                        PrimalEvalEpi<T, false>{v.x, cs, ls, v.xbar, aty, st}, s);
    rb_spmv<double>(A, av, (const T *)v.xbar,
                    DualEvalEpi<T>{v.y, axc, bs, v.ybar, axh, st}, s);
}

#define INST_HALPERN(T)                                                        \
    template void launch_primal_halpern<T>(const DevCsr &, const Iter<T> &,   \
                                           bool, const State *, int,          \
                                           hipStream_t);                      \
    template void launch_dual_halpern<T>(const DevCsr &, const Iter<T> &,     \
                                         const State *, int, hipStream_t);    \
    template void launch_eval_T<T>(const DevCsr &, const DevCsr &,            \
                                   const Iter<T> &, bool, const double *,     \
                                   const double *, const double *,            \
                                   const State *, double *, double *,         \
                                   const double *, hipStream_t);
INST_HALPERN(double)
INST_HALPERN(float)
#undef INST_HALPERN

template void launch_primal<double>(const DevCsr &, const Iter<double> &, bool,
                                    bool, const State *, int, hipStream_t);
template void launch_primal<float>(const DevCsr &, const Iter<float> &, bool,
                                   bool, const State *, int, hipStream_t);
template void launch_dual<double>(const DevCsr &, const Iter<double> &, bool,
                                  const State *, int, hipStream_t);
template void launch_dual<float>(const DevCsr &, const Iter<float> &, bool,
                                 const State *, int, hipStream_t);

// ============================================================ adjoint

template <typename T>
void launch_adj_dual_bwd(const DevCsr &At, const T *gy, const T *gx_in,
                         const T *x1, const T *ls, bool has_l, T *gx_out,
                         T *gv, T *gc, double tau, double sigma,
                         hipStream_t s) {
    if (has_l)
        rbT<T>(At, gy, AdjDualEpi<T, true>{gx_in, x1, ls, gx_out, gv, gc, (T)tau, (T)sigma}, s);
    else
        rbT<T>(At, gy, AdjDualEpi<T, false>{gx_in, x1, ls, gx_out, gv, gc, (T)tau, (T)sigma}, s);
}

template <typename T>
void launch_adj_primal_bwd(const DevCsr &A, const T *gv, const T *gy_in,
                           T *gy_out, T *gb, double tau, double sigma,
                           hipStream_t s) {
    rbT<T>(A, gv, AdjPrimalEpi<T>{gy_in, gy_out, gb, (T)tau, (T)sigma}, s);
}

// dA~_p += tau y_k,i gv_j - sigma gy_{k+1},i (2 x_{k+1},j - x_k,j), p = (i, j)
template <typename T>
__global__ __launch_bounds__(kWG) void k_adj_gA(
    const int32_t *__restrict__ rowidx, const int32_t *__restrict__ ci,
    int64_t nnz, const T *__restrict__ y0, const T *__restrict__ gy1,
    const T *__restrict__ gv, const T *__restrict__ x0,
    const T *__restrict__ x1, T *__restrict__ gA, T tau, T sigma) {
    for (int64_t p = blockIdx.x * (int64_t)kWG + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * kWG) {
        const int i = rowidx[p], j = ci[p];
        const T xb = (x1[j] + x1[j]) - x0[j];
        gA[p] = gA[p] + (tau * y0[i] * gv[j] - sigma * gy1[i] * xb);
    }
}

template <typename T>
void launch_adj_gA(const DevCsr &A, const int32_t *rowidx, const T *y0,
                   const T *gy1, const T *gv, const T *x0, const T *x1, T *gA,
                   double tau, double sigma, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_gA<T>, dim3(grid_for(A.nnz, kWG, 16384)),
                       dim3(kWG), 0, s, rowidx, A.ci, A.nnz, y0, gy1, gv, x0,
                       x1, gA, (T)tau, (T)sigma);
}

#define INST_ADJ(T)                                                          \
    template void launch_adj_dual_bwd<T>(const DevCsr &, const T *,         \
                                         const T *, const T *, const T *,   \
                                         bool, T *, T *, T *, double,       \
                                         double, hipStream_t);              \
    template void launch_adj_primal_bwd<T>(const DevCsr &, const T *,       \
                                           const T *, T *, T *, double,     \
                                           double, hipStream_t);            \
    template void launch_adj_gA<T>(const DevCsr &, const int32_t *,         \
                                   const T *, const T *, const T *,         \
                                   const T *, const T *, T *, double,       \
                                   double, hipStream_t);
INST_ADJ(double)
INST_ADJ(float)
#undef INST_ADJ

// ============================================================ KKT evaluation

namespace {

template <typename T>
struct KktArgs {
    const T *x[2], *y[2], *xl, *yl;
    const double *ax[2], *aty[2];
    const double *bs, *cs, *ls, *dr, *dc;
    int64_t m, n;
    int ncand;
};

// Blocks [0, kRedBlocks) reduce over rows, [kRedBlocks, 2 kRedBlocks) over
// columns.  Per candidate c and quantity q the block writes its partial to
// partial[(c * Q_NQ + q) * 2 kRedBlocks + block].
template <typename T>
__global__ __launch_bounds__(kWG) void k_kkt(KktArgs<T> a,
                                            double *__restrict__ partial) {
    __shared__ double s_red[4];
    double acc[2][Q_NQ];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q = 0; q < Q_NQ; ++q) acc[c][q] = 0.0;
    const int blk = blockIdx.x;
    const int64_t stride = (int64_t)kRedBlocks * kWG;
    if (blk < kRedBlocks) {
        for (int64_t i = (int64_t)blk * kWG + threadIdx.x; i < a.m; i += stride) {
            const double bi = a.bs[i], dri = a.dr[i], yli = (double)a.yl[i];
            for (int c = 0; c < a.ncand; ++c) {
                const double rs = bi - a.ax[c][i];
                const double ru = rs / dri;
                acc[c][Q_RP2] += ru * ru;
                acc[c][Q_RPMAX] = fmax(acc[c][Q_RPMAX], fabs(ru));
                acc[c][Q_SRP2] += rs * rs;
                const double yv = (double)a.y[c][i];
                acc[c][Q_BY] += bi * yv;
                const double dy = yv - yli;
                acc[c][Q_DY2] += dy * dy;
            }
            if (a.ncand > 1) {
                const double f = (double)a.y[1][i] - (double)a.y[0][i];
                acc[1][Q_FY2] += f * f;
            }
        }
    } else {
        for (int64_t j = (int64_t)(blk - kRedBlocks) * kWG + threadIdx.x;
             j < a.n; j += stride) {
            const double cj = a.cs[j], dcj = a.dc[j], xlj = (double)a.xl[j];
            const double lj = a.ls ? a.ls[j] : 0.0;
            for (int c = 0; c < a.ncand; ++c) {
                const double ds = cj - a.aty[c][j];
                const double zs = ds > 0.0 ? ds : 0.0;
                const double rds = zs - ds;
                const double du = ds / dcj;
                const double zu = du > 0.0 ? du : 0.0;
                const double rdu = zu - du;
                acc[c][Q_RD2] += rdu * rdu;
                acc[c][Q_RDMAX] = fmax(acc[c][Q_RDMAX], fabs(rdu));
                acc[c][Q_SRD2] += rds * rds;
                const double xv = (double)a.x[c][j];
                acc[c][Q_CX] += cj * xv;
                acc[c][Q_LZ] += lj * zs;
                const double dx = xv - xlj;
                acc[c][Q_DX2] += dx * dx;
            }
            if (a.ncand > 1) {
                const double f = (double)a.x[1][j] - (double)a.x[0][j];
                acc[1][Q_FX2] += f * f;
            }
        }
    }
    const int nb = 2 * kRedBlocks;
    for (int c = 0; c < a.ncand; ++c)
        for (int q = 0; q < Q_NQ; ++q) {
            double v = (q == Q_RPMAX || q == Q_RDMAX) ? block_max(acc[c][q], s_red)
                                                      : block_sum(acc[c][q], s_red);
            if (threadIdx.x == 0) partial[(c * Q_NQ + q) * nb + blk] = v;
        }
}

// One evaluation's decisions: a fixed-order finish of the partial sums in one
// workgroup, then control_decide (control.h) on thread 0.
__global__ __launch_bounds__(kWG) void k_control(State *st,
                                                 const double *__restrict__ partial,
                                                 int ncand, int batch,
                                                 int initial, double *elog) {
    __shared__ double tot[2][Q_NQ];
    __shared__ double sred[kWG];
    __shared__ int running;
    const int tid = threadIdx.x;
    if (tid == 0) running = (st->status == PDHG_RUNNING);
    __syncthreads();
    if (!running) {
        if (tid == 0) {
            st->copy_pending = 0;
            st->snap_n = 0;
        }
        return;
    }
    const int nb = 2 * kRedBlocks;
    for (int c = 0; c < ncand; ++c)
        for (int q = 0; q < Q_NQ; ++q) {
            const bool isMax = (q == Q_RPMAX || q == Q_RDMAX);
            double v = 0.0;
            for (int b = tid; b < nb; b += kWG) {
                const double p = partial[(c * Q_NQ + q) * nb + b];
                v = isMax ? fmax(v, p) : v + p;
            }
            sred[tid] = v;
            __syncthreads();
            for (int s = kWG / 2; s > 0; s >>= 1) {
                if (tid < s)
                    sred[tid] = isMax ? fmax(sred[tid], sred[tid + s])
                                      : sred[tid] + sred[tid + s];
                __syncthreads();
            }
            if (tid == 0) tot[c][q] = sred[0];
            __syncthreads();
        }
    if (tid == 0) control_decide(st, tot, ncand, batch, initial, elog);
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_polish_stash(
    const State *st, const T *x0, const T *y0, const T *x1, const T *y1,
    const double *dr, const double *dc, double *xs, double *ys, int64_t m,
    int64_t n) {
    if (!st->polish_due) return;
    const T *x = st->polish_cand ? x1 : x0;
    const T *y = st->polish_cand ? y1 : y0;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x; j < n; j += stride)
        xs[j] = dc[j] * (double)x[j];
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < m; i += stride)
        ys[i] = dr[i] * (double)y[i];
}

__global__ void k_advance(State *st, int batch) {
    if (threadIdx.x == 0 && st->status == PDHG_RUNNING) {
        st->k += batch;
        st->t_base += batch;
        st->copy_pending = 0;
        st->snap_n = 0;
    }
}

__global__ void k_set_status(State *st, int status) {
    if (threadIdx.x == 0 && st->status == PDHG_RUNNING) {
        st->status = status;
        st->copy_pending = 0;
        st->snap_n = 0;
    }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_restart_apply(
    const State *__restrict__ st, T *x, T *y, T *ax, T *xbar, T *ybar,
    const double *ax_avg, T *xl, T *yl, T *ax0, int64_t m, int64_t n) {
    if (!st->copy_pending) return;
    const bool avg = st->copy_avg != 0, last = st->set_last != 0;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    // a restart also starts the averages afresh (from zero, so that the first
    // average after it is exactly the first iterate)
    for (int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x; j < n; j += stride) {
        const T v = avg ? xbar[j] : x[j];
        if (avg) x[j] = v;
        if (last) {
            xl[j] = v;
            xbar[j] = (T)0;
        }
    }
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < m; i += stride) {
        const T v = avg ? ybar[i] : y[i];
        if (avg) {
            y[i] = v;
            ax[i] = (T)ax_avg[i];
        }
        if (last) {
            yl[i] = v;
            ybar[i] = (T)0;
            if (ax0) ax0[i] = avg ? (T)ax_avg[i] : ax[i];
        }
    }
}

// Unscaled snapshot of candidate snap_cand into slot snap_first:
// x = D_c x~, y = D_r y~, z = max(0, (c~ - A~^T y~) / D_c).
template <typename T>
__global__ __launch_bounds__(kWG) void k_snapshot_pack(
    const State *__restrict__ st, const T *x0, const T *y0, const T *x1,
    const T *y1, const double *aty0, const double *aty1, const double *cs,
    const double *dr, const double *dc, const int32_t *pr, const int32_t *pc,
    double *slots, int64_t m, int64_t n) {
    if (st->snap_n == 0) return;
    const int c = st->snap_cand;
    const T *x = c ? x1 : x0;
    const T *y = c ? y1 : y0;
    const double *aty = c ? aty1 : aty0;
    double *base = slots + (int64_t)st->snap_first * (2 * n + m);
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x; j < n; j += stride) {
        const int64_t o = pc[j];
        base[o] = dc[j] * (double)x[j];
        const double d = (cs[j] - aty[j]) / dc[j];
        base[n + m + o] = d > 0.0 ? d : 0.0;
    }
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < m; i += stride)
        base[n + pr[i]] = dr[i] * (double)y[i];
}

}  // namespace

void launch_kkt_reduce(int ncand, const void *x0, const void *y0,
                       const void *x1, const void *y1, bool f32,
                       const double *ax0, const double *aty0,
                       const double *ax1, const double *aty1, const void *xl,
                       const void *yl, const double *bs, const double *cs,
                       const double *ls, const double *dr, const double *dc,
                       int64_t m, int64_t n, double *partial, hipStream_t s) {
    if (f32) {
        KktArgs<float> a{{(const float *)x0, (const float *)x1},
                         {(const float *)y0, (const float *)y1},
                         (const float *)xl, (const float *)yl,
                         {ax0, ax1}, {aty0, aty1}, bs, cs, ls, dr, dc, m, n,
                         ncand};
        hipLaunchKernelGGL(k_kkt<float>, dim3(2 * kRedBlocks), dim3(kWG), 0,
                           s, a, partial);
    } else {
        KktArgs<double> a{{(const double *)x0, (const double *)x1},
                          {(const double *)y0, (const double *)y1},
                          (const double *)xl, (const double *)yl,
                          {ax0, ax1}, {aty0, aty1}, bs, cs, ls, dr, dc, m, n,
                          ncand};
        hipLaunchKernelGGL(k_kkt<double>, dim3(2 * kRedBlocks), dim3(kWG), 0,
                           s, a, partial);
    }
}

void launch_control(State *st, const double *partial, int ncand, int batch,
                    int initial, double *log, hipStream_t s) {
    hipLaunchKernelGGL(k_control, dim3(1), dim3(kWG), 0, s, st, partial,
                       ncand, batch, initial, log);
}

void launch_polish_stash(const State *st, bool f32, const void *x0,
                         const void *y0, const void *x1, const void *y1,
                         const double *dr, const double *dc, double *xs,
                         double *ys, int64_t m, int64_t n, hipStream_t s) {
    const int g = grid_for(n > m ? n : m, kWG, 4096);
    if (f32)
        hipLaunchKernelGGL(k_polish_stash<float>, dim3(g), dim3(kWG), 0, s, st,
                           (const float *)x0, (const float *)y0, (const float *)x1,
                           (const float *)y1, dr, dc, xs, ys, m, n);
    else
        hipLaunchKernelGGL(k_polish_stash<double>, dim3(g), dim3(kWG), 0, s, st,
                           (const double *)x0, (const double *)y0,
                           (const double *)x1, (const double *)y1, dr, dc, xs,
                           ys, m, n);
}

void launch_advance(State *st, int batch, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, st, batch);
}

void launch_set_status(State *st, int status, hipStream_t s) {
    hipLaunchKernelGGL(k_set_status, dim3(1), dim3(64), 0, s, st, status);
}

void launch_restart_apply(State *st, bool f32, void *x, void *y, void *ax,
                          void *xbar, void *ybar, const double *ax_avg,
                          void *xl, void *yl, void *ax0, int64_t m, int64_t n,
                          hipStream_t s) {
    const int g = grid_for(n > m ? n : m, kWG, 4096);
    if (f32)
        hipLaunchKernelGGL(k_restart_apply<float>, dim3(g), dim3(kWG), 0, s,
                           st, (float *)x, (float *)y, (float *)ax,
                           (float *)xbar, (float *)ybar, ax_avg,
                           (float *)xl, (float *)yl, (float *)ax0, m, n);
    else
        hipLaunchKernelGGL(k_restart_apply<double>, dim3(g), dim3(kWG), 0, s,
                           st, (double *)x, (double *)y, (double *)ax,
                           (double *)xbar, (double *)ybar, ax_avg,
                           (double *)xl, (double *)yl, (double *)ax0, m, n);
}

void launch_snapshot_pack(const State *st, bool f32, const void *x0,
                          const void *y0, const void *x1, const void *y1,
                          const double *aty0, const double *aty1,
                          const double *cs, const double *dr, const double *dc,
                          const int32_t *pr, const int32_t *pc, double *slots,
                          int64_t m, int64_t n, hipStream_t s) {
    const int g = grid_for(n > m ? n : m, kWG, 4096);
    if (f32)
        hipLaunchKernelGGL(k_snapshot_pack<float>, dim3(g), dim3(kWG), 0, s,
                           st, (const float *)x0, (const float *)y0,
                           (const float *)x1, (const float *)y1, aty0, aty1,
                           cs, dr, dc, pr, pc, slots, m, n);
    else
        hipLaunchKernelGGL(k_snapshot_pack<double>, dim3(g), dim3(kWG), 0, s,
                           st, (const double *)x0, (const double *)y0,
                           (const double *)x1, (const double *)y1, aty0, aty1,
                           cs, dr, dc, pr, pc, slots, m, n);
}

// ============================================================ Ruiz scaling

namespace {

// G lanes per row; rho_r = max over the row of |(rs * v) * cs| where for the
// rows of A (transposed = 0) rs = d_row[r], cs = d_col[ci]; for the rows of
// A^T (transposed = 1) the first factor is the column's: (d_col[ci] * v) *
// d_row[r].  Both orders are (D_r,i * a_ij) * D_c,j for entry (i, j).
template <int G>
__global__ __launch_bounds__(kWG) void k_ruiz_rowmax(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const double *__restrict__ v, const double *__restrict__ d_row,
    const double *__restrict__ d_col, int transposed, int64_t rows,
    double *__restrict__ rho) {
    const int64_t g = ((int64_t)blockIdx.x * kWG + threadIdx.x) / G;
    const int lane = threadIdx.x & (G - 1);
    const int64_t ngroups = (int64_t)gridDim.x * kWG / G;
    // every lane runs the same number of rounds so the shuffles are uniform
    for (int64_t base = 0; base < rows; base += ngroups) {
        const int64_t r = base + g;
        double mx = 0.0;
        if (r < rows) {
            const double dr = d_row[r];
            for (int p = rp[r] + lane; p < rp[r + 1]; p += G) {
                const double a = transposed ? (d_col[ci[p]] * v[p]) * dr
                                            : (dr * v[p]) * d_col[ci[p]];
                mx = fmax(mx, fabs(a));
            }
        }
        for (int o = G >> 1; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
        if (r < rows && lane == 0) rho[r] = mx;
    }
}

__global__ __launch_bounds__(kWG) void k_ruiz_update(double *d,
                                                     const double *rho,
                                                     int64_t k) {
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * kWG) {
        double r = rho[i];
        if (r == 0.0) r = 1.0;
        d[i] = d[i] / sqrt(r);
    }
}

template <int G>
__global__ __launch_bounds__(kWG) void k_scale_values(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const double *__restrict__ v, const double *__restrict__ d_row,
    const double *__restrict__ d_col, int transposed, int64_t rows,
    double *__restrict__ out, float *__restrict__ out32) {
    const int64_t g = ((int64_t)blockIdx.x * kWG + threadIdx.x) / G;
    const int lane = threadIdx.x & (G - 1);
    const int64_t ngroups = (int64_t)gridDim.x * kWG / G;
    for (int64_t r = g; r < rows; r += ngroups) {
        const double dr = d_row[r];
        for (int p = rp[r] + lane; p < rp[r + 1]; p += G) {
            const double a = transposed ? (d_col[ci[p]] * v[p]) * dr
                                        : (dr * v[p]) * d_col[ci[p]];
            out[p] = a;
            if (out32) out32[p] = (float)a;
        }
    }
}

int lanes_for(const DevCsr &M) {
    const double avg = M.rows ? (double)M.nnz / (double)M.rows : 1.0;
    if (avg <= 4) return 4;
    if (avg <= 8) return 8;
    if (avg <= 16) return 16;
    if (avg <= 32) return 32;
    return 64;
}

}  // namespace

void launch_ruiz_rowmax(const DevCsr &M, const double *d_row,
                        const double *d_col, int transposed, double *rho,
                        hipStream_t s) {
    const int G = lanes_for(M);
    const int g = grid_for(M.rows * G, kWG, 16384);
    switch (G) {
        case 4: hipLaunchKernelGGL(k_ruiz_rowmax<4>, dim3(g), dim3(kWG), 0, s, M.rp, M.ci, M.v_orig, d_row, d_col, transposed, M.rows, rho); break;
        case 8: hipLaunchKernelGGL(k_ruiz_rowmax<8>, dim3(g), dim3(kWG), 0, s, M.rp, M.ci, M.v_orig, d_row, d_col, transposed, M.rows, rho); break;
        case 16: hipLaunchKernelGGL(k_ruiz_rowmax<16>, dim3(g), dim3(kWG), 0, s, M.rp, M.ci, M.v_orig, d_row, d_col, transposed, M.rows, rho); break;
        case 32: hipLaunchKernelGGL(k_ruiz_rowmax<32>, dim3(g), dim3(kWG), 0, s, M.rp, M.ci, M.v_orig, d_row, d_col, transposed, M.rows, rho); break;
        default: hipLaunchKernelGGL(k_ruiz_rowmax<64>, dim3(g), dim3(kWG), 0, s, M.rp, M.ci, M.v_orig, d_row, d_col, transposed, M.rows, rho); break;
    }
}

void launch_ruiz_update(double *d, const double *rho, int64_t k,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_ruiz_update, dim3(grid_for(k, kWG, 4096)), dim3(kWG),
                       0, s, d, rho, k);
}

void launch_scale_values(const DevCsr &M, const double *v, const double *rs,
                         const double *cs, double *out, float *out32,
                         hipStream_t s) {
    const int G = lanes_for(M);
    const int g = grid_for(M.rows * G, kWG, 16384);
    switch (G) {
        case 4: hipLaunchKernelGGL(k_scale_values<4>, dim3(g), dim3(kWG), 0, s, M.rp, M.ci, v, rs, cs, 0, M.rows, out, out32); break;
        case 8: hipLaunchKernelGGL(k_scale_values<8>, dim3(g), dim3(kWG), 0, s, M.rp, M.ci, v, rs, cs, 0, M.rows, out, out32); break;
        case 16: hipLaunchKernelGGL(k_scale_values<16>, dim3(g), dim3(kWG), 0, s, M.rp, M.ci, v, rs, cs, 0, M.rows, out, out32); break;
        case 32: hipLaunchKernelGGL(k_scale_values<32>, dim3(g), dim3(kWG), 0, s, M.rp, M.ci, v, rs, cs, 0, M.rows, out, out32); break;
        default: hipLaunchKernelGGL(k_scale_values<64>, dim3(g), dim3(kWG), 0, s, M.rp, M.ci, v, rs, cs, 0, M.rows, out, out32); break;
    }
}

// ============================================================ vector kernels

namespace {

__global__ __launch_bounds__(kWG) void k_dot_partial(const double *a,
                                                     const double *b,
                                                     int64_t k,
                                                     double *partial) {
    __shared__ double s_red[4];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * kWG)
        acc += a[i] * b[i];
    acc = block_sum(acc, s_red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// mode 0: sum of partials; mode 1: max of partials
__global__ __launch_bounds__(kWG) void k_finish(const double *partial, int np,
                                                double *result, int mode) {
    __shared__ double sred[kWG];
    const int tid = threadIdx.x;
    double v = 0.0;
    for (int b = tid; b < np; b += kWG)
        v = mode ? fmax(v, partial[b]) : v + partial[b];
    sred[tid] = v;
    __syncthreads();
    for (int s = kWG / 2; s > 0; s >>= 1) {
        if (tid < s)
            sred[tid] = mode ? fmax(sred[tid], sred[tid + s])
                             : sred[tid] + sred[tid + s];
        __syncthreads();
    }
    if (tid == 0) *result = sred[0];
}

// dst = src / sqrt(*factor) (mode 0) ; dst = src * (*factor) (mode 1)
__global__ __launch_bounds__(kWG) void k_scale_vec(double *dst,
                                                   const double *src,
                                                   const double *factor,
                                                   int64_t k, int mode) {
    const double f = *factor;
    const double nrm = sqrt(f);
    if (mode == 0 && !(nrm > 0.0)) {
        for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < k;
             i += (int64_t)gridDim.x * kWG)
            dst[i] = src[i];
        return;
    }
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * kWG)
        dst[i] = mode == 0 ? src[i] / nrm : src[i] * f;
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_fill(T *p, T v, int64_t k) {
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * kWG)
        p[i] = v;
}

template <typename D, typename S>
__global__ __launch_bounds__(kWG) void k_convert(D *dst, const S *src,
                                                 int64_t k) {
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * kWG)
        dst[i] = (D)src[i];
}

__global__ __launch_bounds__(kWG) void k_ew(double *out, const double *a,
                                            const double *b, int64_t k,
                                            int mode) {
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * kWG) {
        if (mode == 0)
            out[i] = a[i] * b[i];
        else if (mode == 1)
            out[i] = a[i] / b[i];
        else
            out[i] = a[i] * b[0];
    }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_unscale_xyz(
    const T *xs, const T *ys, const double *aty, const double *cs,
    const double *dr, const double *dc, const int32_t *pr, const int32_t *pc,
    double *x, double *y, double *z, int64_t m, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x; j < n; j += stride) {
        const int64_t o = pc[j];
        if (x) x[o] = dc[j] * (double)xs[j];
        if (z) {
            const double d = (cs[j] - aty[j]) / dc[j];
            z[o] = d > 0.0 ? d : 0.0;
        }
    }
    if (y)
        for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < m; i += stride)
            y[pr[i]] = dr[i] * (double)ys[i];
}

__global__ __launch_bounds__(kWG) void k_gather(double *dst,
                                                const double *src,
                                                const int32_t *idx,
                                                int64_t k) {
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * kWG)
        dst[i] = src[idx[i]];
}

__global__ __launch_bounds__(kWG) void k_permute(double *dst,
                                                 const double *src,
                                                 const int32_t *perm,
                                                 int64_t k) {
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * kWG)
        dst[perm[i]] = src[i];
}

// Correction LP data in the scaled space: b^ = DP (b~ - A~x~),
// c^ = DD (c~ - A~^T y~), l^ = -DP x~.
__global__ __launch_bounds__(kWG) void k_refine_rhs(
    const double *bs, const double *ax, const double *cs, const double *aty,
    const double *xs, const double *ls, double DP, double DD, double *bh,
    double *ch, double *lh, int64_t m, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < m; i += stride)
        bh[i] = DP * (bs[i] - ax[i]);
    for (int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x; j < n; j += stride) {
        ch[j] = DD * (cs[j] - aty[j]);
        lh[j] = DP * ((ls ? ls[j] : 0.0) - xs[j]);
    }
}

// Per block: max |r_P,i| and max (l_j - x_j)^+ (unscaled) into
// partial[0][b], max (-d_j)^+ into partial[1][b].
__global__ __launch_bounds__(kWG) void k_refine_delta(
    const double *bs, const double *ax, const double *cs, const double *aty,
    const double *xs, const double *ls, const double *dr, const double *dc,
    int64_t m, int64_t n, double *partial) {
    __shared__ double s_red[4];
    double dp = 0.0, dd = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < m; i += stride)
        dp = fmax(dp, fabs((bs[i] - ax[i]) / dr[i]));
    for (int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x; j < n; j += stride) {
        dp = fmax(dp, dc[j] * ((ls ? ls[j] : 0.0) - xs[j]));
        dd = fmax(dd, -((cs[j] - aty[j]) / dc[j]));
    }
    dp = block_max(dp, s_red);
    dd = block_max(dd, s_red);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = dp;
        partial[gridDim.x + blockIdx.x] = dd;
    }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_refine_update(
    double *xs, double *ys, const T *xh, const T *yh, const double *ls,
    double invP, double invD, int64_t m, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t j = (int64_t)blockIdx.x * kWG + threadIdx.x; j < n; j += stride) {
        const double v = xs[j] + (double)xh[j] * invP;
        const double lj = ls ? ls[j] : 0.0;
        xs[j] = v < lj ? lj : v;
    }
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < m; i += stride)
        ys[i] = ys[i] + (double)yh[i] * invD;
}

__global__ __launch_bounds__(kWG) void k_norm_unscaled_partial(
    const double *vs, const double *d, int64_t k, double *partial) {
    __shared__ double s_red[4];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * kWG) {
        const double u = vs[i] / d[i];
        acc += u * u;
    }
    acc = block_sum(acc, s_red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

}  // namespace

void launch_dot(const double *a, const double *b, int64_t k, double *partial,
                double *result, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(kWG), 0, s, a, b,
                       k, partial);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kWG), 0, s, partial,
                       kRedBlocks, result, 0);
}

void launch_norm_unscaled(const double *vs, const double *d, int64_t k,
                          double *partial, double *result, hipStream_t s) {
    hipLaunchKernelGGL(k_norm_unscaled_partial, dim3(kRedBlocks), dim3(kWG),
                       0, s, vs, d, k, partial);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kWG), 0, s, partial,
                       kRedBlocks, result, 0);
}

void launch_scale_vec(double *dst, const double *src, const double *factor,
                      int64_t k, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_vec, dim3(grid_for(k, kWG, 4096)), dim3(kWG), 0,
                       s, dst, src, factor, k, mode);
}

void launch_fill(double *p, double v, int64_t k, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(k, kWG, 4096)),
                       dim3(kWG), 0, s, p, v, k);
}

void launch_fill32(float *p, float v, int64_t k, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(k, kWG, 4096)), dim3(kWG),
                       0, s, p, v, k);
}

void launch_to_f32(float *dst, const double *src, int64_t k, hipStream_t s) {
    hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_for(k, kWG, 4096)),
                       dim3(kWG), 0, s, dst, src, k);
}

void launch_to_f64(double *dst, const float *src, int64_t k, hipStream_t s) {
    hipLaunchKernelGGL((k_convert<double, float>), dim3(grid_for(k, kWG, 4096)),
                       dim3(kWG), 0, s, dst, src, k);
}

void launch_ew(double *out, const double *a, const double *b, int64_t k,
               int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_ew, dim3(grid_for(k, kWG, 4096)), dim3(kWG), 0, s,
                       out, a, b, k, mode);
}

void launch_unscale_xyz(const double *xs, const double *ys, const double *aty,
                        const double *cs, const double *dr, const double *dc,
                        const int32_t *pr, const int32_t *pc, double *x,
                        double *y, double *z, int64_t m, int64_t n,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_unscale_xyz<double>,
                       dim3(grid_for(n > m ? n : m, kWG, 4096)), dim3(kWG), 0,
                       s, xs, ys, aty, cs, dr, dc, pr, pc, x, y, z, m, n);
}

void launch_unscale_xyz32(const float *xs, const float *ys, const double *aty,
                          const double *cs, const double *dr,
                          const double *dc, const int32_t *pr,
                          const int32_t *pc, double *x, double *y, double *z,
                          int64_t m, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_unscale_xyz<float>,
                       dim3(grid_for(n > m ? n : m, kWG, 4096)), dim3(kWG), 0,
                       s, xs, ys, aty, cs, dr, dc, pr, pc, x, y, z, m, n);
}

void launch_permute(double *dst, const double *src, const int32_t *perm,
                    int64_t k, hipStream_t s) {
    hipLaunchKernelGGL(k_permute, dim3(grid_for(k, kWG, 16384)), dim3(kWG), 0,
                       s, dst, src, perm, k);
}

void launch_gather(double *dst, const double *src, const int32_t *idx,
                   int64_t k, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3(grid_for(k, kWG, 16384)), dim3(kWG), 0,
                       s, dst, src, idx, k);
}

void launch_refine_rhs(const double *bs, const double *ax, const double *cs,
                       const double *aty, const double *xs, const double *ls,
                       double DP, double DD, double *bh, double *ch,
                       double *lh, int64_t m, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_refine_rhs, dim3(grid_for(n > m ? n : m, kWG, 4096)),
                       dim3(kWG), 0, s, bs, ax, cs, aty, xs, ls, DP, DD, bh,
                       ch, lh, m, n);
}

void launch_refine_delta(const double *bs, const double *ax, const double *cs,
                         const double *aty, const double *xs,
                         const double *ls, const double *dr, const double *dc,
                         int64_t m, int64_t n, double *partial, double *out2,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_refine_delta, dim3(kRedBlocks), dim3(kWG), 0, s, bs,
                       ax, cs, aty, xs, ls, dr, dc, m, n, partial);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kWG), 0, s, partial,
                       kRedBlocks, out2, 1);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kWG), 0, s,
                       partial + kRedBlocks, kRedBlocks, out2 + 1, 1);
}

template <typename T>
void launch_refine_update(double *xs, double *ys, const T *xh, const T *yh,
                          const double *ls, double DP, double DD, int64_t m,
                          int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_refine_update<T>,
                       dim3(grid_for(n > m ? n : m, kWG, 4096)), dim3(kWG), 0,
                       s, xs, ys, xh, yh, ls, 1.0 / DP, 1.0 / DD, m, n);
}
template void launch_refine_update<float>(double *, double *, const float *,
                                          const float *, const double *,
                                          double, double, int64_t, int64_t,
                                          hipStream_t);
template void launch_refine_update<double>(double *, double *, const double *,
                                           const double *, const double *,
                                           double, double, int64_t, int64_t,
                                           hipStream_t);

// ============================================================ gather probe

namespace {

// splitmix64 finaliser (Steele, Lea and Flood's SplitMix generator): a
// counter-based hash giving the probe its random indices.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Indices of the probe's stream: entry i belongs to workgroup i / chunk,
// which gathers only from its panel (w % 8) % P of the table, as the row
// blocks of a panelled SpMV side do (workgroup w runs on XCD w % 8).
__global__ __launch_bounds__(kWG) void k_probe_fill(int32_t *idx, int64_t n,
                                                    int64_t chunk,
                                                    int64_t table, int P,
                                                    uint64_t seed) {
    const int64_t stride = (int64_t)gridDim.x * kWG;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) {
        const int64_t w = i / chunk;
        const int p = (int)((w % 8) % P);
        const int64_t lo = table * p / P, hi = table * (p + 1) / P;
        idx[i] = (int32_t)(lo + (int64_t)(mix64(seed + (uint64_t)i) % (uint64_t)(hi - lo)));
    }
}

// The SpMV's memory pattern without the row structure: workgroup w streams
// the (index, value) pairs [w chunk, (w + 1) chunk) with 16-byte loads, four
// per thread at a time, gathers table[index] for each and sums the products.
template <typename T, bool NT>
__global__ __launch_bounds__(kWG) void k_gather_probe(const int32_t *idx,
                                                      const T *val,
                                                      const T *table,
                                                      int64_t chunk,
                                                      int64_t n, T *out) {
    __shared__ T sred[4];
    const int64_t b0 = (int64_t)blockIdx.x * chunk;
    const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
    T acc = 0;
    for (int64_t p = b0 + 4 * (int64_t)threadIdx.x; p < b1; p += 4 * kWG) {
        int j[4];
        T a[4];
        ld4<NT>(idx + p, j);
        ld4<NT>(val + p, a);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (p + q < b1) acc += a[q] * table[j[q]];
    }
    acc = block_sum(acc, sred);
    if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

}  // namespace

void launch_probe_fill(int32_t *idx, int64_t n, int64_t chunk, int64_t table,
                       int P, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_probe_fill, dim3(grid_for(n, kWG, 16384)), dim3(kWG),
                       0, s, idx, n, chunk, table, P, seed);
}

template <typename T>
void launch_gather_probe(const int32_t *idx, const T *val, const T *table,
                         int64_t chunk, int64_t n, bool nt, T *out,
                         hipStream_t s) {
    const int g = (int)((n + chunk - 1) / chunk);
    if (nt)
        hipLaunchKernelGGL((k_gather_probe<T, true>), dim3(g), dim3(kWG), 0, s,
                           idx, val, table, chunk, n, out);
    else
        hipLaunchKernelGGL((k_gather_probe<T, false>), dim3(g), dim3(kWG), 0, s,
                           idx, val, table, chunk, n, out);
}
template void launch_gather_probe<double>(const int32_t *, const double *,
                                          const double *, int64_t, int64_t,
                                          bool, double *, hipStream_t);
template void launch_gather_probe<float>(const int32_t *, const float *,
                                         const float *, int64_t, int64_t,
                                         bool, float *, hipStream_t);

}  // namespace pdhg
