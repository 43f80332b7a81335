// pdhg.cpp -- host side of libpdhg.so: the C ABI declared in include/pdhg.h.
//
// The context owns every device buffer.  Problem data live on the device in
// both FP64 and FP32; the iterate lives in the precision of the bulk
// iteration.  The host only launches kernels and reads back, once per
// evaluation, the small control state that the device-side control kernel
// writes (status, snapshot levels fired, restart counters).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "job_queue.h"

using namespace pdhg;

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct DevError {
    int code;
    std::string msg;
};

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        std::string m = std::string(what) + ": " + hipGetErrorString(e);
        throw DevError{e == hipErrorOutOfMemory ? PDHG_E_OOM : PDHG_E_DEVICE, m};
    }
}

#define HIPC(call) hip_check((call), #call)

template <typename T>
T *dmalloc(int64_t count) {
    if (count <= 0) count = 1;
    void *p = nullptr;
    hip_check(hipMalloc(&p, (size_t)count * sizeof(T)), "hipMalloc");
    return (T *)p;
}

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

struct ProfRec {
    int kind;  // 0 primal, 1 dual
    hipEvent_t a, b;
};

struct SnapMeta {
    pdhg_snapshot_info info;
    int slot;
};

struct CbItem {
    int idx;
    int slot;                   // host copy the callback reads
    hipEvent_t ev;
    pdhg_snapshot_info info;    // copied at enqueue: the list may grow meanwhile
    // taken at enqueue, under the callback lock: the slot table may be
    // resized and the callback replaced while the item waits
    const double *host;
    pdhg_snapshot_cb cb;
    void *user;
};

}  // namespace

// Device scratch of the allocation-free SpMV (pdhg_spmv_noalloc): one copy per
// GPU, held from module load until the process ends.  Host code never uses
// this name as an address; it uses the per-device pointer that
// hipGetSymbolAddress returns (scratch_ptr below).
constexpr size_t kScratchBytes = PDHG_SPMV_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of `scratch` on `device`, looked up once per device with
// that device current.
void *scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices)
        throw DevError{PDHG_E_DEVICE, "device ordinal beyond the scratch table"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                  "hipGetSymbolAddress(scratch)");
        if (!p) throw DevError{PDHG_E_DEVICE, "null scratch address"};
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}

}  // namespace

struct pdhg_ctx {
    int device = 0;
    void *scratch = nullptr;    // this device's copy of `scratch` (device address)
    hipStream_t stream = nullptr, copy_stream = nullptr;
    bool own_stream = false;
    std::string err;

    // problem
    bool loaded = false, configured = false;
    int64_t m = 0, n = 0, nnz = 0;
    DevCsr A, At;
    // internal relabeling (rows and columns by decreasing length)
    int32_t *pr = nullptr;      // internal row -> original row of A
    int32_t *pc = nullptr;      // internal column -> original column
    int32_t *apos = nullptr;    // internal nonzero -> position in A's arrays
    int32_t *perm = nullptr;    // A' position -> A'^T position
    int32_t *rowidx = nullptr;  // row of each of A''s nonzeros
    double *tmp_m = nullptr, *tmp_n = nullptr;  // staging for I/O
    double *b_orig = nullptr, *c_orig = nullptr, *l_orig = nullptr;
    bool has_l = false;
    int64_t split_threshold = (int64_t)1 << 20;
    int64_t split_chunk = (int64_t)1 << 16;
    int panels_a = 0, panels_at = 0;    // column panels per side; 0 = choose
    int stream_nt = -1;                 // streamed-load kind; -1 = choose
    int sort_rows = -1, sort_cols = -1; // length sort of rows / columns; -1 = by skew
    int block_rows = kWG;               // row cap of multi-row blocks; 0 = tile

    // scaling and scaled data
    double *dr = nullptr, *dc = nullptr;
    double *bs = nullptr, *cs = nullptr, *ls = nullptr;       // FP64
    float *bs32 = nullptr, *cs32 = nullptr, *ls32 = nullptr;  // FP32
    // refinement correction data
    double *bh = nullptr, *ch = nullptr, *lh = nullptr;
    float *bh32 = nullptr, *ch32 = nullptr, *lh32 = nullptr;
    double *xo = nullptr, *yo = nullptr;  // outer FP64 iterate (scaled)

    // feasibility polishing: the candidate set aside (unscaled), the phase
    // results (scaled), zero data vectors, and the main solve's iterate
    double *pol_x = nullptr, *pol_y = nullptr, *pol_xp = nullptr, *pol_yd = nullptr;
    double *zero_n = nullptr, *zero_m = nullptr;
    float *zero_n32 = nullptr, *zero_m32 = nullptr;
    Iter<double> bk64;
    Iter<float> bk32;
    int polish_attempts = 0;
    int64_t polish_iters = 0;

    // active problem of the current solve
    const double *act_bs = nullptr, *act_cs = nullptr, *act_ls = nullptr;
    bool act_has_l = false;

    Iter<double> v64;
    Iter<float> v32;
    int prec = PDHG_FP64;

    // evaluation temporaries
    double *aty_cur = nullptr, *aty_avg = nullptr, *ax_avg = nullptr,
           *ax_cur = nullptr;
    double *partial = nullptr, *scal = nullptr, *rho = nullptr, *kap = nullptr;
    double *log = nullptr;
    int log_cap = 4096;
    double *slots = nullptr;
    int n_slots = 0;

    State *st = nullptr;       // device
    State *st_host = nullptr;  // pinned
    State st_init;

    pdhg_params params;
    std::vector<double> levels;
    double sigma_hat = 0, eta = 0, omega0 = 0;
    double nb = 0, nc = 0;

    // host bookkeeping of a solve
    bool initial_done = false;
    int64_t k_host = 0;
    int status = PDHG_RUNNING;
    double t_setup = 0, t_iter = 0, t_start = 0;
    std::atomic<int> cancel_flag{0};
    std::vector<SnapMeta> snaps;
    bool keep_snaps = false;        // refinement: inner solves keep the list
    bool keep_cancel = false;       // refinement: inner solves keep a cancel
    std::function<void(int)> snap_hook;   // new snapshots [arg, end) recorded
    std::vector<double> refine_log;   // 10 doubles per refinement round
    // outer-progress test of a refinement inner solve (active when set):
    // the round's outer iterate, scales and target; the best refined point
    // its evaluations have seen (FP64, scaled), its maxresid and iteration;
    // the stall window and whether the round was ended for stalling
    const double *ref_xo = nullptr, *ref_yo = nullptr;
    double ref_DP = 1.0, ref_DD = 1.0, ref_target = -1.0;
    double *ref_bx = nullptr, *ref_by = nullptr;
    double ref_best = INFINITY;
    int64_t ref_best_k = 0, ref_stall = 0;
    bool ref_cut = false;

    // callback thread
    pdhg_snapshot_cb cb = nullptr;
    void *cb_user = nullptr;
    std::thread cb_thread;
    std::mutex cb_mu;
    std::condition_variable cb_cv;
    std::condition_variable cb_done_cv;   // a slot's callbacks have all run
    std::deque<CbItem> cb_queue;
    bool cb_stop = false;
    std::vector<double *> host_snap;      // pinned host copy per slot
    std::vector<int> host_snap_busy;      // queued or running callbacks per slot

    // graphs: one per (precision, eval_every, active pointers)
    hipGraphExec_t graph = nullptr;
    std::vector<const void *> graph_key;

    // live adjoint tapes (detached when the context is destroyed)
    std::vector<pdhg_tape *> tapes;
    // generation of the problem data an adjoint replay reads (structure,
    // values, b, c, l, scaling, relabeling): bumped by load, configure,
    // set_values and set_rhs_obj; a tape records it at its forward pass
    uint64_t data_gen = 0;

    // profiling
    bool profile = false;
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> ev_pool;
    int64_t prof_launch[2] = {0, 0};
    double prof_ms[2] = {0, 0};
};

struct pdhg_tape {
    pdhg_ctx *ctx = nullptr;
    uint64_t data_gen = 0;      // the context's data_gen at the forward pass
    int K = 0, ck = 0, prec = PDHG_FP64, nseg = 0;
    double tau = 0, sigma = 0;
    void *ckx = nullptr, *cky = nullptr, *ckax = nullptr;
    State *st = nullptr;
};

extern "C" {
static void tape_release(pdhg_tape *tp);
}

namespace {

int fail(pdhg_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

#define API_BEGIN(ctx)                               \
    if (!(ctx)) return PDHG_E_ARG;                   \
    (ctx)->err.clear();                              \
    try {                                            \
        hip_check(hipSetDevice((ctx)->device), "hipSetDevice");
#define API_END(ctx)                                 \
    }                                                \
    catch (const DevError &e) {                      \
        return fail((ctx), e.code, e.msg);           \
    }                                                \
    catch (const std::bad_alloc &) {                 \
        return fail((ctx), PDHG_E_OOM, "host allocation failed"); \
    }                                                \
    catch (...) {                                    \
        return fail((ctx), PDHG_E_DEVICE, "unexpected exception"); \
    }

// Copy `count` elements into a device buffer from host or device memory.
template <typename T>
void copy_in(pdhg_ctx *c, T *dst, const T *src, int64_t count, int mem) {
    if (count <= 0) return;
    hip_check(hipMemcpyAsync(dst, src, (size_t)count * sizeof(T),
                             mem == PDHG_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                    : hipMemcpyHostToDevice,
                             c->stream),
              "hipMemcpyAsync(in)");
}

template <typename T>
void copy_out(pdhg_ctx *c, T *dst, const T *src, int64_t count, int mem) {
    if (count <= 0 || !dst) return;
    hip_check(hipMemcpyAsync(dst, src, (size_t)count * sizeof(T),
                             mem == PDHG_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                    : hipMemcpyDeviceToHost,
                             c->stream),
              "hipMemcpyAsync(out)");
}

void sync(pdhg_ctx *c) { HIPC(hipStreamSynchronize(c->stream)); }

// Caller vector in original order -> internal order (dst[i'] = src[idx[i']]).
void vec_in(pdhg_ctx *c, double *dst, const double *src, bool rows, int mem) {
    const int64_t k = rows ? c->m : c->n;
    double *tmp = rows ? c->tmp_m : c->tmp_n;
    copy_in(c, tmp, src, k, mem);
    launch_gather(dst, tmp, rows ? c->pr : c->pc, k, c->stream);
}

// Internal vector -> caller buffer in original order.
void vec_out(pdhg_ctx *c, double *dst, const double *src, bool rows, int mem) {
    if (!dst) return;
    const int64_t k = rows ? c->m : c->n;
    double *tmp = rows ? c->tmp_m : c->tmp_n;
    launch_permute(tmp, src, rows ? c->pr : c->pc, k, c->stream);
    copy_out(c, dst, tmp, k, mem);
}

// Device staging of one pdhg_spmv call: the input and output in internal
// order, and their FP32 copies for the FP32 kernel.
struct SpmvStage {
    double *din = nullptr, *dout = nullptr;
    float *i32 = nullptr, *o32 = nullptr;
};

// Bytes of SpmvStage for a side with `cols` inputs and `rows` outputs, each
// array rounded up to 256 bytes.
size_t spmv_noalloc_bytes(int64_t cols, int64_t rows, int precision) {
    auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t b = r((size_t)cols * 8) + r((size_t)rows * 8);
    if (precision == PDHG_FP32) b += r((size_t)cols * 4) + r((size_t)rows * 4);
    return b;
}

// FP32 values of M (and of its panel copy, whose FP64 values are rewritten
// from the same source) rounded from `vals` (nnz, M's order).
void put_f32_values(pdhg_ctx *c, const DevCsr &M, const double *vals) {
    launch_to_f32(M.v32, vals, M.nnz, c->stream);
    if (M.pan) {
        launch_gather(M.pan->v64, vals, M.pan_src, M.nnz, c->stream);
        launch_to_f32(M.pan->v32, M.pan->v64, M.nnz, c->stream);
    }
}

// out = M in for M = A (which 0) or A^T (which 1), through the staging
// buffers st: gather `in` into internal order, run the binned SpMV kernel of
// the requested precision, scatter back to the caller's order.  Returns
// after the stream has finished.
void spmv_staged(pdhg_ctx *c, int which, int scaled, int precision,
                 const double *in, double *out, int mem, const SpmvStage &st) {
    const DevCsr &M = which ? c->At : c->A;
    vec_in(c, st.din, in, which == 1, mem);
    if (precision == PDHG_FP32) {
        launch_to_f32(st.i32, st.din, M.cols, c->stream);
        // the FP32 kernel reads M.v32 (or its panel copy): put the loaded
        // values there for an unscaled product, restore the scaled ones after
        if (!scaled) put_f32_values(c, M, M.v_orig);
        spmv_f32(M, st.i32, st.o32, c->stream);
        launch_to_f64(st.dout, st.o32, M.rows, c->stream);
        if (!scaled) put_f32_values(c, M, M.v64);
    } else {
        spmv_f64(M, scaled ? M.v64 : M.v_orig, st.din, st.dout, c->stream);
    }
    vec_out(c, out, st.dout, which == 0, mem);
    sync(c);
}

// A caller array given by pointer and `mem`, staged to the host when needed.
template <typename T>
std::vector<T> to_host(pdhg_ctx *c, const T *p, int64_t count, int mem) {
    std::vector<T> h((size_t)(count > 0 ? count : 0));
    if (count <= 0) return h;
    if (mem == PDHG_MEM_DEVICE) {
        HIPC(hipMemcpyAsync(h.data(), p, (size_t)count * sizeof(T),
                            hipMemcpyDeviceToHost, c->stream));
        sync(c);
    } else {
        std::memcpy(h.data(), p, (size_t)count * sizeof(T));
    }
    return h;
}

void free_csr(DevCsr &M) {
    if (M.pan) {
        free_csr(*M.pan);
        delete M.pan;
    }
    dfree(M.pan_src);
    dfree(M.pan_mask);
    dfree(M.q64);
    dfree(M.q32);
    dfree(M.rp);
    dfree(M.ci);
    dfree(M.v_orig);
    dfree(M.v64);
    dfree(M.v32);
    dfree(M.blk64);
    dfree(M.blk32);
    dfree(M.split64);
    dfree(M.split32);
    dfree(M.part64);
    dfree(M.part32);
    M = DevCsr();
}

template <typename T>
void free_iter(Iter<T> &v) {
    dfree(v.x);
    dfree(v.y);
    dfree(v.xbar);
    dfree(v.ybar);
    dfree(v.xl);
    dfree(v.yl);
    dfree(v.ax);
    dfree(v.ax0);
}

void invalidate_graph(pdhg_ctx *c) {
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
    c->graph_key.clear();
}

void free_problem(pdhg_ctx *c) {
    // tapes recorded on the data being dropped can no longer be replayed:
    // free their device memory now (their handles stay valid for
    // pdhg_tape_free, and pdhg_unrolled_backward refuses them)
    ++c->data_gen;
    for (pdhg_tape *tp : c->tapes) tape_release(tp);
    invalidate_graph(c);
    free_csr(c->A);
    free_csr(c->At);
    dfree(c->perm);
    dfree(c->rowidx);
    dfree(c->pr);
    dfree(c->pc);
    dfree(c->apos);
    dfree(c->tmp_m);
    dfree(c->tmp_n);
    dfree(c->b_orig);
    dfree(c->c_orig);
    dfree(c->l_orig);
    dfree(c->dr);
    dfree(c->dc);
    dfree(c->bs);
    dfree(c->cs);
    dfree(c->ls);
    dfree(c->bs32);
    dfree(c->cs32);
    dfree(c->ls32);
    dfree(c->bh);
    dfree(c->ch);
    dfree(c->lh);
    dfree(c->bh32);
    dfree(c->ch32);
    dfree(c->lh32);
    dfree(c->xo);
    dfree(c->yo);
    dfree(c->ref_bx);
    dfree(c->ref_by);
    for (double **p : {&c->pol_x, &c->pol_y, &c->pol_xp, &c->pol_yd, &c->zero_n, &c->zero_m})
        dfree(*p);
    dfree(c->zero_n32);
    dfree(c->zero_m32);
    free_iter(c->bk64);
    free_iter(c->bk32);
    free_iter(c->v64);
    free_iter(c->v32);
    dfree(c->aty_cur);
    dfree(c->aty_avg);
    dfree(c->ax_avg);
    dfree(c->ax_cur);
    dfree(c->partial);
    dfree(c->scal);
    dfree(c->rho);
    dfree(c->kap);
    dfree(c->log);
    dfree(c->slots);
    c->n_slots = 0;
    {
        // callbacks still queued or running read the host copies
        std::unique_lock<std::mutex> lk(c->cb_mu);
        c->cb_done_cv.wait(lk, [c] {
            for (int b : c->host_snap_busy)
                if (b) return false;
            return true;
        });
    }
    for (double *h : c->host_snap)
        if (h) (void)hipHostFree(h);
    c->host_snap.clear();
    c->host_snap_busy.clear();
    c->loaded = c->configured = false;
}

void upload_bins(DevCsr &M, const HostBins &b64, const HostBins &b32) {
    M.nblk64 = (int)b64.blocks.size();
    M.nblk32 = (int)b32.blocks.size();
    M.blk64 = dmalloc<RowBlock>(M.nblk64);
    M.blk32 = dmalloc<RowBlock>(M.nblk32);
    if (M.nblk64) HIPC(hipMemcpy(M.blk64, b64.blocks.data(), M.nblk64 * sizeof(RowBlock), hipMemcpyHostToDevice));
    if (M.nblk32) HIPC(hipMemcpy(M.blk32, b32.blocks.data(), M.nblk32 * sizeof(RowBlock), hipMemcpyHostToDevice));
    M.nsplit64 = (int)b64.splits.size();
    M.nsplit32 = (int)b32.splits.size();
    M.maxparts64 = b64.maxparts;
    M.maxparts32 = b32.maxparts;
    M.split64 = dmalloc<SplitRow>(M.nsplit64);
    M.split32 = dmalloc<SplitRow>(M.nsplit32);
    if (M.nsplit64) HIPC(hipMemcpy(M.split64, b64.splits.data(), M.nsplit64 * sizeof(SplitRow), hipMemcpyHostToDevice));
    if (M.nsplit32) HIPC(hipMemcpy(M.split32, b32.splits.data(), M.nsplit32 * sizeof(SplitRow), hipMemcpyHostToDevice));
    M.part64 = dmalloc<double>((int64_t)M.nsplit64 * M.maxparts64);
    M.part32 = dmalloc<float>((int64_t)M.nsplit32 * M.maxparts32);
    for (int q = 0; q < 3; ++q) M.counts64[q] = b64.counts[q];
}

// Index and value arrays padded (zeros) to a multiple of 4 plus 4, so the
// kernels' aligned 16-byte group loads stay inside the allocation.
int64_t padded(int64_t nnz) { return ((nnz + 3) & ~(int64_t)3) + 4; }

// The panel twin of M (P > 1): the stacked panel matrix with its own index
// array and scaled values (filled by apply_scaling), XCD-dealt bins, and the
// P * rows partial sums.
void upload_panels(pdhg_ctx *c, DevCsr &M, const std::vector<int64_t> &rp,
                   const std::vector<int32_t> &ci, int P,
                   const std::vector<int64_t> &cut) {
    Panels S = build_panels(M.rows, rp.data(), ci.data(), P, cut);
    M.P = P;
    M.pan = new DevCsr();
    DevCsr &T = *M.pan;
    T.rows = (int64_t)P * M.rows;
    T.cols = M.cols;
    T.nnz = M.nnz;
    const int64_t pad = padded(M.nnz);
    std::vector<int32_t> rp32((size_t)T.rows + 1);
    for (int64_t i = 0; i <= T.rows; ++i) rp32[i] = (int32_t)S.rp[i];
    T.rp = dmalloc<int32_t>(T.rows + 1);
    T.ci = dmalloc<int32_t>(pad);
    T.v64 = dmalloc<double>(pad);
    T.v32 = dmalloc<float>(pad);
    HIPC(hipMemset(T.ci, 0, pad * sizeof(int32_t)));
    HIPC(hipMemset(T.v64, 0, pad * sizeof(double)));
    HIPC(hipMemset(T.v32, 0, pad * sizeof(float)));
    HIPC(hipMemcpy(T.rp, rp32.data(), (T.rows + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    M.pan_src = dmalloc<int32_t>(M.nnz);
    if (M.nnz) {
        HIPC(hipMemcpy(T.ci, S.ci.data(), M.nnz * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPC(hipMemcpy(M.pan_src, S.src.data(), M.nnz * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    upload_bins(T, build_panel_blocks(M.rows, S.rp.data(), P, kTile64 - 3, c->split_threshold, c->split_chunk, c->block_rows),
                build_panel_blocks(M.rows, S.rp.data(), P, kTile32 - 3, c->split_threshold, c->split_chunk, c->block_rows));
    // the mask is needed only when some row misses some panel
    const uint8_t full = (uint8_t)((1u << P) - 1);
    if (std::any_of(S.mask.begin(), S.mask.end(), [&](uint8_t k) { return k != full; })) {
        M.pan_mask = dmalloc<uint8_t>(M.rows);
        HIPC(hipMemcpy(M.pan_mask, S.mask.data(), M.rows * sizeof(uint8_t), hipMemcpyHostToDevice));
    }
    M.q64 = dmalloc<double>(T.rows);
    M.q32 = dmalloc<float>(T.rows);
}

// Upload one CSR (int64 row pointers on the host) and build both bin sets;
// with P > 1 also its panel twin.
void upload_csr(pdhg_ctx *c, DevCsr &M, int64_t rows, int64_t cols,
                int64_t nnz, const std::vector<int64_t> &rp,
                const std::vector<int32_t> &ci, const std::vector<double> &v,
                int P, const std::vector<int64_t> &cut) {
    M.rows = rows;
    M.cols = cols;
    M.nnz = nnz;
    std::vector<int32_t> rp32((size_t)rows + 1);
    for (int64_t i = 0; i <= rows; ++i) rp32[i] = (int32_t)rp[i];
    const int64_t pad = padded(nnz);
    M.rp = dmalloc<int32_t>(rows + 1);
    M.ci = dmalloc<int32_t>(pad);
    M.v_orig = dmalloc<double>(pad);
    M.v64 = dmalloc<double>(pad);
    M.v32 = dmalloc<float>(pad);
    HIPC(hipMemset(M.ci, 0, pad * sizeof(int32_t)));
    HIPC(hipMemset(M.v_orig, 0, pad * sizeof(double)));
    HIPC(hipMemset(M.v64, 0, pad * sizeof(double)));
    HIPC(hipMemset(M.v32, 0, pad * sizeof(float)));
    HIPC(hipMemcpy(M.rp, rp32.data(), (rows + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    if (nnz > 0) {
        HIPC(hipMemcpy(M.ci, ci.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPC(hipMemcpy(M.v_orig, v.data(), nnz * sizeof(double), hipMemcpyHostToDevice));
    }
    // multi-row blocks hold at most TILE - 3 nonzeros: an aligned window of
    // TILE entries then always covers them
    upload_bins(M, build_row_blocks(rows, rp.data(), kTile64 - 3, c->split_threshold, c->split_chunk, c->block_rows),
                build_row_blocks(rows, rp.data(), kTile32 - 3, c->split_threshold, c->split_chunk, c->block_rows));
    if (P > 1) upload_panels(c, M, rp, ci, P, cut);
    // stream the CSR non-temporally when the FP64 gather table each XCD
    // works on exceeds 3 MiB, so that streaming does not evict it from L2
    M.stream_nt = c->stream_nt >= 0 ? c->stream_nt
                                    : (8.0 * (double)cols / P > 3.0 * 1048576.0);
}

template <typename T>
void alloc_iter(Iter<T> &v, int64_t m, int64_t n) {
    if (v.x) return;
    v.x = dmalloc<T>(n);
    v.xbar = dmalloc<T>(n);
    v.xl = dmalloc<T>(n);
    v.y = dmalloc<T>(m);
    v.ybar = dmalloc<T>(m);
    v.yl = dmalloc<T>(m);
    v.ax = dmalloc<T>(m);
    v.ax0 = dmalloc<T>(m);
}

template <typename T>
void zero_iter(pdhg_ctx *c, Iter<T> &v) {
    HIPC(hipMemsetAsync(v.x, 0, c->n * sizeof(T), c->stream));
    HIPC(hipMemsetAsync(v.xbar, 0, c->n * sizeof(T), c->stream));
    HIPC(hipMemsetAsync(v.xl, 0, c->n * sizeof(T), c->stream));
    HIPC(hipMemsetAsync(v.y, 0, c->m * sizeof(T), c->stream));
    HIPC(hipMemsetAsync(v.ybar, 0, c->m * sizeof(T), c->stream));
    HIPC(hipMemsetAsync(v.yl, 0, c->m * sizeof(T), c->stream));
    HIPC(hipMemsetAsync(v.ax, 0, c->m * sizeof(T), c->stream));
    HIPC(hipMemsetAsync(v.ax0, 0, c->m * sizeof(T), c->stream));
}

double read_scalar(pdhg_ctx *c, const double *dptr) {
    double h = 0;
    HIPC(hipMemcpyAsync(&h, dptr, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    return h;
}

double dev_norm(pdhg_ctx *c, const double *v, int64_t k) {
    launch_dot(v, v, k, c->partial, c->scal, c->stream);
    return std::sqrt(read_scalar(c, c->scal));
}

// Scaled values of both CSRs from A's loaded values and the factors.
void apply_scaling(pdhg_ctx *c) {
    launch_scale_values(c->A, c->A.v_orig, c->dr, c->dc, c->A.v64, c->A.v32, c->stream);
    launch_permute(c->At.v64, c->A.v64, c->perm, c->nnz, c->stream);
    launch_to_f32(c->At.v32, c->At.v64, c->nnz, c->stream);
    for (DevCsr *M : {&c->A, &c->At})
        if (M->pan) {
            launch_gather(M->pan->v64, M->v64, M->pan_src, c->nnz, c->stream);
            launch_to_f32(M->pan->v32, M->pan->v64, c->nnz, c->stream);
        }
}

void apply_rhs_scaling(pdhg_ctx *c) {
    launch_ew(c->bs, c->dr, c->b_orig, c->m, 0, c->stream);
    launch_ew(c->cs, c->dc, c->c_orig, c->n, 0, c->stream);
    if (c->has_l) launch_ew(c->ls, c->l_orig, c->dc, c->n, 1, c->stream);
    launch_to_f32(c->bs32, c->bs, c->m, c->stream);
    launch_to_f32(c->cs32, c->cs, c->n, c->stream);
    if (c->has_l) launch_to_f32(c->ls32, c->ls, c->n, c->stream);
    c->nb = dev_norm(c, c->b_orig, c->m);
    c->nc = dev_norm(c, c->c_orig, c->n);
}

void ruiz(pdhg_ctx *c, int passes) {
    launch_fill(c->dr, 1.0, c->m, c->stream);
    launch_fill(c->dc, 1.0, c->n, c->stream);
    for (int p = 0; p < passes; ++p) {
        // row maxima of A and of A^T (the column maxima of A), both from the
        // factors of the previous pass, then both updates
        launch_ruiz_rowmax(c->A, c->dr, c->dc, 0, c->rho, c->stream);
        launch_ruiz_rowmax(c->At, c->dc, c->dr, 1, c->kap, c->stream);
        launch_ruiz_update(c->dr, c->rho, c->m, c->stream);
        launch_ruiz_update(c->dc, c->kap, c->n, c->stream);
    }
}

// Power iteration for sigma_hat ~ ||A~||_2: v0 = 1/sqrt(n) ones, `iters`
// steps of w = A~^T A~ v, v = w / ||w||, then sqrt(||A~^T A~ v||).
double power_iteration(pdhg_ctx *c, int iters) {
    double *v = c->aty_avg, *u = c->ax_avg, *w = c->aty_cur;
    launch_fill(v, 1.0 / std::sqrt((double)c->n), c->n, c->stream);
    for (int it = 0; it <= iters; ++it) {
        spmv_f64(c->A, c->A.v64, v, u, c->stream);
        spmv_f64(c->At, c->At.v64, u, w, c->stream);
        launch_dot(w, w, c->n, c->partial, c->scal, c->stream);
        if (it < iters) launch_scale_vec(v, w, c->scal, c->n, 0, c->stream);
    }
    double nw2 = read_scalar(c, c->scal);
    double s = std::sqrt(std::sqrt(nw2));
    return (s > 0.0 && std::isfinite(s)) ? s : 1.0;
}

void write_state(pdhg_ctx *c, const State &s) {
    HIPC(hipMemcpyAsync(c->st, &s, sizeof(State), hipMemcpyHostToDevice, c->stream));
    sync(c);
}

void read_state(pdhg_ctx *c) {
    HIPC(hipMemcpyAsync(c->st_host, c->st, sizeof(State), hipMemcpyDeviceToHost, c->stream));
    sync(c);
}

// Initial control state for a fresh solve of the active problem.
State fresh_state(pdhg_ctx *c, double omega, double nb, double nc) {
    State s;
    std::memset(&s, 0, sizeof s);
    s.eta = c->eta;
    s.omega = omega;
    s.tau = c->eta / omega;
    s.sigma = c->eta * omega;
    s.K_last = INFINITY;
    s.K_prev = INFINITY;
    s.nb = nb;
    s.nc = nc;
    s.eps_rel = c->params.eps_rel;
    s.beta_suff = c->params.beta_suff;
    s.beta_nec = c->params.beta_nec;
    s.beta_art = c->params.beta_art;
    s.omega_theta = c->params.omega_theta;
    s.omega_rule = c->params.omega_rule;
    s.pid_kp = c->params.pid_kp;
    s.pid_ki = c->params.pid_ki;
    s.pid_kd = c->params.pid_kd;
    s.pid_int = 0.0;
    s.pid_eprev = 0.0;
    s.stop_on = c->params.stop_on;
    s.polish = c->params.polish;
    s.next_polish = 0;
    s.variant = c->params.variant;
    s.reflect = c->params.reflect;
    s.status = PDHG_RUNNING;
    s.n_levels = (int)c->levels.size();
    s.literal = c->params.literal_snapshots;
    s.log_cap = c->log_cap;
    for (size_t i = 0; i < c->levels.size(); ++i) s.levels[i] = c->levels[i];
    return s;
}

void reset_solve(pdhg_ctx *c) {
    c->initial_done = false;
    c->k_host = 0;
    c->status = PDHG_RUNNING;
    c->t_iter = 0;
    if (!c->keep_snaps) c->snaps.clear();
    if (!c->keep_cancel) c->cancel_flag.store(0);
}

bool f32(pdhg_ctx *c) { return c->prec == PDHG_FP32; }

void *cur_x(pdhg_ctx *c) { return f32(c) ? (void *)c->v32.x : (void *)c->v64.x; }
void *cur_y(pdhg_ctx *c) { return f32(c) ? (void *)c->v32.y : (void *)c->v64.y; }

// A~ x and A~^T y (FP64) of the current iterate into ax_cur / aty_cur.
void current_products(pdhg_ctx *c, bool need_ax) {
    if (f32(c)) {
        if (need_ax) spmv_f64_in32(c->A, c->A.v64, c->v32.x, c->ax_cur, c->stream);
        spmv_f64_in32(c->At, c->At.v64, c->v32.y, c->aty_cur, c->stream);
    } else {
        if (need_ax) spmv_f64(c->A, c->A.v64, c->v64.x, c->ax_cur, c->stream);
        spmv_f64(c->At, c->At.v64, c->v64.y, c->aty_cur, c->stream);
    }
}

// The evaluation sequence after a batch of `batch` iterations (initial: the
// k = 0 check of the starting point, current iterate only).
void enqueue_eval(pdhg_ctx *c, int batch, bool initial) {
    const bool h = f32(c);
    const bool halpern = c->params.variant == 1;
    const int ncand = (initial && !halpern) ? 1 : 2;
    // FP64 products of the candidates
    if (halpern) {
        // candidate 1 is T(z), computed here in FP64 arithmetic
        const double *bs = c->act_bs, *cs = c->act_cs;
        const double *ls = c->act_has_l ? c->act_ls : nullptr;
        if (h) {
            spmv_f64_in32(c->A, c->A.v64, c->v32.x, c->ax_cur, c->stream);
            launch_eval_T<float>(c->A, c->At, c->v32, c->act_has_l, cs, bs, ls,
                                 c->st, c->aty_cur, c->ax_avg, c->ax_cur, c->stream);
            spmv_f64_in32(c->At, c->At.v64, c->v32.ybar, c->aty_avg, c->stream);
        } else {
            launch_eval_T<double>(c->A, c->At, c->v64, c->act_has_l, cs, bs, ls,
                                  c->st, c->aty_cur, c->ax_avg, c->v64.ax, c->stream);
            spmv_f64(c->At, c->At.v64, c->v64.ybar, c->aty_avg, c->stream);
        }
    } else if (h) {
        spmv_f64_in32(c->A, c->A.v64, c->v32.x, c->ax_cur, c->stream);
        spmv_f64_in32(c->At, c->At.v64, c->v32.y, c->aty_cur, c->stream);
        if (!initial) {
            spmv_f64_in32(c->A, c->A.v64, c->v32.xbar, c->ax_avg, c->stream);
            spmv_f64_in32(c->At, c->At.v64, c->v32.ybar, c->aty_avg, c->stream);
        }
    } else {
        spmv_f64(c->At, c->At.v64, c->v64.y, c->aty_cur, c->stream);
        if (!initial) {
            spmv_f64(c->A, c->A.v64, c->v64.xbar, c->ax_avg, c->stream);
            spmv_f64(c->At, c->At.v64, c->v64.ybar, c->aty_avg, c->stream);
        }
    }
    const double *axc = h ? c->ax_cur : c->v64.ax;
    const void *x0 = h ? (void *)c->v32.x : (void *)c->v64.x;
    const void *y0 = h ? (void *)c->v32.y : (void *)c->v64.y;
    const void *x1 = h ? (void *)c->v32.xbar : (void *)c->v64.xbar;
    const void *y1 = h ? (void *)c->v32.ybar : (void *)c->v64.ybar;
    const void *xl = h ? (void *)c->v32.xl : (void *)c->v64.xl;
    const void *yl = h ? (void *)c->v32.yl : (void *)c->v64.yl;
    launch_kkt_reduce(ncand, x0, y0, x1, y1, h, axc, c->aty_cur, c->ax_avg,
                      c->aty_avg, xl, yl, c->act_bs, c->act_cs,
                      c->act_has_l ? c->act_ls : nullptr, c->dr, c->dc, c->m,
                      c->n, c->partial, c->stream);
    launch_control(c->st, c->partial, ncand, batch, initial ? 1 : 0, c->log,
                   c->stream);
    if (c->n_slots > 0)
        launch_snapshot_pack(c->st, h, x0, y0, x1, y1, c->aty_cur, c->aty_avg,
                             c->act_cs, c->dr, c->dc, c->pr, c->pc, c->slots,
                             c->m, c->n, c->stream);
    if (c->params.polish)
        launch_polish_stash(c->st, h, x0, y0, x1, y1, c->dr, c->dc, c->pol_x,
                            c->pol_y, c->m, c->n, c->stream);
    if (h)
        launch_restart_apply(c->st, true, c->v32.x, c->v32.y, c->v32.ax,
                             c->v32.xbar, c->v32.ybar, c->ax_avg, c->v32.xl,
                             c->v32.yl, halpern ? (void *)c->v32.ax0 : nullptr,
                             c->m, c->n, c->stream);
    else
        launch_restart_apply(c->st, false, c->v64.x, c->v64.y, c->v64.ax,
                             c->v64.xbar, c->v64.ybar, c->ax_avg, c->v64.xl,
                             c->v64.yl, halpern ? (void *)c->v64.ax0 : nullptr,
                             c->m, c->n, c->stream);
    if (h) spmv_f32(c->A, c->v32.x, c->v32.ax, c->stream);
}

hipEvent_t pool_event(pdhg_ctx *c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPC(hipEventCreate(&e));
    return e;
}

void enqueue_iterations(pdhg_ctx *c, int first_off, int count) {
    for (int off = first_off; off < first_off + count; ++off) {
        ProfRec r0{0, nullptr, nullptr}, r1{1, nullptr, nullptr};
        if (c->profile) {
            r0.a = pool_event(c);
            r0.b = pool_event(c);
            HIPC(hipEventRecord(r0.a, c->stream));
        }
        const bool halpern = c->params.variant == 1;
        if (halpern && f32(c))
            launch_primal_halpern<float>(c->At, c->v32, c->act_has_l, c->st, off, c->stream);
        else if (halpern)
            launch_primal_halpern<double>(c->At, c->v64, c->act_has_l, c->st, off, c->stream);
        else if (f32(c))
            launch_primal<float>(c->At, c->v32, c->act_has_l, true, c->st, off, c->stream);
        else
            launch_primal<double>(c->At, c->v64, c->act_has_l, true, c->st, off, c->stream);
        if (c->profile) {
            HIPC(hipEventRecord(r0.b, c->stream));
            r1.a = pool_event(c);
            r1.b = pool_event(c);
            HIPC(hipEventRecord(r1.a, c->stream));
        }
        if (halpern && f32(c))
            launch_dual_halpern<float>(c->A, c->v32, c->st, off, c->stream);
        else if (halpern)
            launch_dual_halpern<double>(c->A, c->v64, c->st, off, c->stream);
        else if (f32(c))
            launch_dual<float>(c->A, c->v32, true, c->st, off, c->stream);
        else
            launch_dual<double>(c->A, c->v64, true, c->st, off, c->stream);
        if (c->profile) {
            HIPC(hipEventRecord(r1.b, c->stream));
            c->prof.push_back(r0);
            c->prof.push_back(r1);
        }
    }
}

void resolve_profile(pdhg_ctx *c) {
    if (c->prof.empty()) return;
    sync(c);
    for (auto &r : c->prof) {
        float ms = 0;
        HIPC(hipEventElapsedTime(&ms, r.a, r.b));
        c->prof_ms[r.kind] += ms;
        c->prof_launch[r.kind] += 1;
        c->ev_pool.push_back(r.a);
        c->ev_pool.push_back(r.b);
    }
    c->prof.clear();
}

std::vector<const void *> current_graph_key(pdhg_ctx *c) {
    return {(const void *)(intptr_t)c->prec, (const void *)(intptr_t)c->params.eval_every,
            (const void *)(intptr_t)c->params.variant,
            c->act_bs, c->act_cs, c->act_ls, (const void *)(intptr_t)c->act_has_l,
            cur_x(c), (const void *)(intptr_t)c->n_slots};
}

// One full batch (eval_every iterations + evaluation) as a replayed graph.
bool launch_batch_graph(pdhg_ctx *c) {
    auto key = current_graph_key(c);
    if (!c->graph || key != c->graph_key) {
        invalidate_graph(c);
        hipGraph_t g;
        HIPC(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        enqueue_iterations(c, 0, c->params.eval_every);
        enqueue_eval(c, c->params.eval_every, false);
        HIPC(hipStreamEndCapture(c->stream, &g));
        hipError_t e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->graph = nullptr;
            hip_check(e, "hipGraphInstantiate");
        }
        c->graph_key = key;
    }
    HIPC(hipGraphLaunch(c->graph, c->stream));
    return true;
}

void cb_worker(pdhg_ctx *c) {
    for (;;) {
        CbItem it;
        {
            std::unique_lock<std::mutex> lk(c->cb_mu);
            c->cb_cv.wait(lk, [c] { return c->cb_stop || !c->cb_queue.empty(); });
            if (c->cb_queue.empty()) return;
            it = c->cb_queue.front();
            c->cb_queue.pop_front();
        }
        (void)hipEventSynchronize(it.ev);
        (void)hipEventDestroy(it.ev);
        if (it.cb) it.cb(it.user, it.idx, &it.info, it.host, it.host + c->n, it.host + c->n + c->m);
        {
            std::lock_guard<std::mutex> lk(c->cb_mu);
            --c->host_snap_busy[it.slot];
        }
        c->cb_done_cv.notify_all();
    }
}

void start_snapshot_copies(pdhg_ctx *c, int before);

// New snapshots reported by the last evaluation: record their metadata and,
// when a callback is registered, start their host copy on the copy stream.
void collect_snapshots(pdhg_ctx *c) {
    const State &s = *c->st_host;
    const int before = (int)c->snaps.size();
    for (int i = before; i < s.snap_count; ++i) {
        SnapMeta sm;
        std::memset(&sm, 0, sizeof sm);
        sm.info.level = s.snap_level[i];
        sm.info.iter = s.snap_iter[i];
        sm.info.maxresid = s.snap_mr[i];
        sm.info.candidate = s.snap_cand_of[i];
        sm.info.t_wall = now_s() - c->t_start;
        sm.slot = s.snap_first;
        c->snaps.push_back(sm);
    }
    start_snapshot_copies(c, before);
    if (c->snap_hook && (int)c->snaps.size() > before) c->snap_hook(before);
}

// Snapshots [before, end) share the slot of the first: copy it to pinned host
// memory on the copy stream and queue their callbacks behind the copy.
void start_snapshot_copies(pdhg_ctx *c, int before) {
    {
        std::lock_guard<std::mutex> lk(c->cb_mu);
        if (!c->cb) return;
    }
    if ((int)c->snaps.size() == before) return;
    const int64_t len = 2 * c->n + c->m;
    const int slot = c->snaps[before].slot;
    {
        // the slot's host copy is rewritten only after the callbacks still
        // reading it (from an earlier solve) have returned
        std::unique_lock<std::mutex> lk(c->cb_mu);
        // (during refinement n_slots is 0 for the inner solves: size by the slot)
        if ((int)c->host_snap.size() <= slot) {
            c->host_snap.resize(slot + 1, nullptr);
            c->host_snap_busy.resize(slot + 1, 0);
        }
        c->cb_done_cv.wait(lk, [c, slot] { return c->host_snap_busy[slot] == 0; });
    }
    double *host = nullptr;
    {
        std::lock_guard<std::mutex> lk(c->cb_mu);
        host = c->host_snap[slot];
    }
    if (!host) {
        HIPC(hipHostMalloc((void **)&host, len * sizeof(double), hipHostMallocDefault));
        std::lock_guard<std::mutex> lk(c->cb_mu);
        c->host_snap[slot] = host;
    }
    hipEvent_t ready, done;
    HIPC(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    HIPC(hipEventRecord(ready, c->stream));
    HIPC(hipStreamWaitEvent(c->copy_stream, ready, 0));
    HIPC(hipMemcpyAsync(host, c->slots + (int64_t)slot * len,
                        len * sizeof(double), hipMemcpyDeviceToHost, c->copy_stream));
    HIPC(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    HIPC(hipEventRecord(done, c->copy_stream));
    (void)hipEventDestroy(ready);
    {
        std::lock_guard<std::mutex> lk(c->cb_mu);
        for (int i = before; i < (int)c->snaps.size(); ++i) {
            hipEvent_t e = done;
            if (i > before) {
                HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
                HIPC(hipEventRecord(e, c->copy_stream));
            }
            c->cb_queue.push_back({i, slot, e, c->snaps[i].info, host, c->cb, c->cb_user});
            ++c->host_snap_busy[slot];
        }
    }
    c->cb_cv.notify_one();
}

void kkt_pair64(pdhg_ctx *c, const double *xs, const double *ys,
                const double *bs, const double *cs, const double *ls,
                double nb, double nc, pdhg_kkt *out);

// Refinement: has the refined point max(l, xo + x^/DP), yo + y^/DD of the
// current inner iterate reached the round's target on the original LP?
template <typename T>
bool refine_outer_reached_T(pdhg_ctx *c, Iter<T> &v) {
    // the Halpern variant reports T(z) (left in xbar / ybar by the
    // evaluation) unless a restart has just made it the current iterate
    const bool th = c->params.variant == 1 &&
                    !(c->st_host->copy_pending && c->st_host->set_last);
    const T *xi = th ? v.xbar : v.x;
    const T *yi = th ? v.ybar : v.y;
    const double *ls = c->has_l ? c->ls : nullptr;
    HIPC(hipMemcpyAsync(c->xo, c->ref_xo, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPC(hipMemcpyAsync(c->yo, c->ref_yo, c->m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    launch_refine_update<T>(c->xo, c->yo, xi, yi, ls, c->ref_DP, c->ref_DD, c->m, c->n, c->stream);
    pdhg_kkt K;
    kkt_pair64(c, c->xo, c->yo, c->bs, c->cs, ls, c->nb, c->nc, &K);
    if (K.maxresid < c->ref_best) {
        // the best refined point of the round so far
        HIPC(hipMemcpyAsync(c->ref_bx, c->xo, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HIPC(hipMemcpyAsync(c->ref_by, c->yo, c->m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        c->ref_best = K.maxresid;
        c->ref_best_k = c->k_host;
    }
    const bool ok = K.maxresid <= c->ref_target;
    if (ok && th) {
        HIPC(hipMemcpyAsync(v.x, v.xbar, c->n * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
        HIPC(hipMemcpyAsync(v.y, v.ybar, c->m * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
    }
    return ok;
}

bool refine_outer_reached(pdhg_ctx *c) {
    return c->prec == PDHG_FP64 ? refine_outer_reached_T(c, c->v64)
                                : refine_outer_reached_T(c, c->v32);
}

void polish(pdhg_ctx *c);

// The iteration loop shared by pdhg_iterate, the refinement's inner solves
// and the polishing phases.  Runs until the status leaves RUNNING or
// `max_more` iterations.
int run_iterations(pdhg_ctx *c, int64_t max_more, int64_t limit_total) {
    if (!c->initial_done) {
        c->t_start = now_s();
        enqueue_eval(c, 0, true);
        read_state(c);
        c->initial_done = true;
        c->status = c->st_host->status;
        collect_snapshots(c);
    }
    const double t0 = now_s();
    const int64_t target = std::min(c->k_host + max_more, limit_total);
    const int N = c->params.eval_every;
    while (c->status == PDHG_RUNNING) {
        if (c->k_host >= limit_total) {
            launch_set_status(c->st, PDHG_ITER_LIMIT, c->stream);
            read_state(c);
            c->status = c->st_host->status;
            break;
        }
        if (c->k_host >= target) break;
        const int64_t rem = target - c->k_host;
        const int to_eval = N - (int)(c->k_host % N);
        const int B = (int)std::min<int64_t>(rem, to_eval);
        const bool eval = (B == to_eval);
        if (eval && B == N && c->params.use_graph && !c->profile) {
            launch_batch_graph(c);
        } else {
            enqueue_iterations(c, 0, B);
            if (eval)
                enqueue_eval(c, B, false);
            else
                launch_advance(c->st, B, c->stream);
        }
        c->k_host += B;
        if (eval) {
            read_state(c);
            c->status = c->st_host->status;
            c->k_host = c->st_host->k;
            collect_snapshots(c);
            if (c->status == PDHG_RUNNING && c->st_host->polish_due) polish(c);
            if (c->status == PDHG_RUNNING && c->ref_target >= 0.0) {
                if (refine_outer_reached(c)) {
                    launch_set_status(c->st, PDHG_CONVERGED, c->stream);
                    read_state(c);
                    c->status = c->st_host->status;
                } else if (c->ref_stall > 0 &&
                           c->k_host - c->ref_best_k > std::max(c->ref_stall, 4 * c->ref_best_k)) {
                    // the refined point has stopped improving: end the round
                    c->ref_cut = true;
                    launch_set_status(c->st, PDHG_ITER_LIMIT, c->stream);
                    read_state(c);
                    c->status = c->st_host->status;
                }
            }
            if (c->status == PDHG_RUNNING) {
                int stop = 0;
                if (c->cancel_flag.load()) stop = PDHG_CANCELLED;
                else if (c->params.time_limit_s > 0 &&
                         now_s() - c->t_start > c->params.time_limit_s)
                    stop = PDHG_TIME_LIMIT;
                if (stop) {
                    launch_set_status(c->st, stop, c->stream);
                    read_state(c);
                    c->status = c->st_host->status;
                }
            }
            if (c->profile) resolve_profile(c);
        }
    }
    if (c->profile) resolve_profile(c);
    sync(c);
    c->t_iter += now_s() - t0;
    return c->status;
}

void kkt_of(pdhg_ctx *c, int which, pdhg_kkt *out);

void finish_totals(pdhg_ctx *c, const double *Q, double nb, double nc,
                   pdhg_kkt *o) {
    o->norm_rp = std::sqrt(Q[Q_RP2]);
    o->norm_rd = std::sqrt(Q[Q_RD2]);
    o->rp_inf = Q[Q_RPMAX];
    o->rd_inf = Q[Q_RDMAX];
    o->pobj = Q[Q_CX];
    o->dobj = Q[Q_BY] + Q[Q_LZ];
    o->rel_p = o->norm_rp / (1.0 + nb);
    o->rel_d = o->norm_rd / (1.0 + nc);
    o->rel_gap = std::fabs(o->pobj - o->dobj) /
                 (1.0 + std::fabs(o->pobj) + std::fabs(o->dobj));
    o->maxresid = std::max(o->rel_p, std::max(o->rel_d, o->rel_gap));
    if (!std::isfinite(o->rel_p) || !std::isfinite(o->rel_d) || !std::isfinite(o->rel_gap))
        o->maxresid = NAN;
    (void)c;
}

// FP64 KKT of an arbitrary scaled FP64 pair on the active problem, through
// the same reduction kernel as the evaluations (partials then host sums in a
// fixed order).
void kkt_pair64(pdhg_ctx *c, const double *xs, const double *ys,
                const double *bs, const double *cs, const double *ls,
                double nb, double nc, pdhg_kkt *out) {
    spmv_f64(c->A, c->A.v64, xs, c->ax_cur, c->stream);
    spmv_f64(c->At, c->At.v64, ys, c->aty_cur, c->stream);
    launch_kkt_reduce(1, xs, ys, xs, ys, false, c->ax_cur, c->aty_cur,
                      c->ax_cur, c->aty_cur, xs, ys, bs, cs, ls, c->dr, c->dc,
                      c->m, c->n, c->partial, c->stream);
    const int nbk = 2 * kRedBlocks;
    std::vector<double> h((size_t)Q_NQ * nbk);
    HIPC(hipMemcpyAsync(h.data(), c->partial, h.size() * sizeof(double),
                        hipMemcpyDeviceToHost, c->stream));
    sync(c);
    double Q[Q_NQ];
    for (int q = 0; q < Q_NQ; ++q) {
        double v = 0.0;
        for (int b = 0; b < nbk; ++b) {
            double p = h[(size_t)q * nbk + b];
            v = (q == Q_RPMAX || q == Q_RDMAX) ? std::max(v, p) : v + p;
        }
        Q[q] = v;
    }
    finish_totals(c, Q, nb, nc, out);
}

void kkt_of(pdhg_ctx *c, int which, pdhg_kkt *out) {
    // bring the candidate to FP64 scaled vectors in xo/yo scratch
    const bool h = f32(c);
    double *xs = c->xo, *ys = c->yo;
    if (h) {
        launch_to_f64(xs, which ? c->v32.xbar : c->v32.x, c->n, c->stream);
        launch_to_f64(ys, which ? c->v32.ybar : c->v32.y, c->m, c->stream);
    } else {
        HIPC(hipMemcpyAsync(xs, which ? c->v64.xbar : c->v64.x, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HIPC(hipMemcpyAsync(ys, which ? c->v64.ybar : c->v64.y, c->m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    }
    kkt_pair64(c, xs, ys, c->act_bs, c->act_cs, c->act_has_l ? c->act_ls : nullptr,
               c->st_host->nb, c->st_host->nc, out);
    out->iter = c->k_host;
    out->candidate = which;
}

void configure_solve_state(pdhg_ctx *c) {
    c->act_bs = c->bs;
    c->act_cs = c->cs;
    c->act_ls = c->ls;
    c->act_has_l = c->has_l;
    c->v64.bs = c->bs;
    c->v64.cs = c->cs;
    c->v64.ls = c->ls;
    c->v32.bs = c->bs32;
    c->v32.cs = c->cs32;
    c->v32.ls = c->ls32;
}

}  // namespace

// ============================================================== the C ABI

extern "C" {

// Message of the last failed pdhg_create on this thread (there is no
// context to hold it).
static thread_local std::string g_create_err;

const char *pdhg_last_error(const pdhg_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int pdhg_create(int device, void *hip_stream, pdhg_ctx **out) {
    g_create_err.clear();
    if (!out) {
        g_create_err = "null out pointer";
        return PDHG_E_ARG;
    }
    *out = nullptr;
    pdhg_ctx *c = nullptr;
    try {
        c = new pdhg_ctx();
    } catch (...) {
        g_create_err = "host allocation failed";
        return PDHG_E_OOM;
    }
    c->device = device;
    try {
        int count = 0;
        HIPC(hipGetDeviceCount(&count));
        if (device < 0 || device >= count) throw DevError{PDHG_E_ARG, "no such device"};
        HIPC(hipSetDevice(device));
        c->scratch = scratch_ptr(device);
        if (hip_stream) {
            c->stream = (hipStream_t)hip_stream;
        } else {
            // a blocking stream: ordered after work on the null stream, so
            // inputs written there by the caller are complete
            HIPC(hipStreamCreate(&c->stream));
            c->own_stream = true;
        }
        HIPC(hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
        HIPC(hipHostMalloc((void **)&c->st_host, sizeof(State), hipHostMallocDefault));
        std::memset(c->st_host, 0, sizeof(State));
        c->st = dmalloc<State>(1);
    } catch (const DevError &e) {
        g_create_err = e.msg;
        pdhg_destroy(c);
        return e.code == PDHG_E_ARG ? PDHG_E_ARG : PDHG_E_DEVICE;
    } catch (...) {
        g_create_err = "host allocation failed";
        pdhg_destroy(c);
        return PDHG_E_OOM;
    }
    pdhg_params_default(&c->params);
    *out = c;
    return PDHG_OK;
}

static void tape_release(pdhg_tape *tp);

void pdhg_destroy(pdhg_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->copy_stream) (void)hipStreamSynchronize(c->copy_stream);
    // tapes still held by the caller lose their device memory and their
    // context; pdhg_tape_free then only releases the handle
    for (pdhg_tape *tp : c->tapes) {
        tape_release(tp);
        tp->ctx = nullptr;
    }
    c->tapes.clear();
    if (c->cb_thread.joinable()) {
        {
            std::lock_guard<std::mutex> lk(c->cb_mu);
            c->cb_stop = true;
        }
        c->cb_cv.notify_all();
        c->cb_thread.join();
    }
    free_problem(c);
    for (auto &r : c->prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    dfree(c->st);
    if (c->st_host) (void)hipHostFree(c->st_host);
    if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int pdhg_set_tuning(pdhg_ctx *c, const char *key, int64_t value) {
    if (!c || !key) return PDHG_E_ARG;
    if (std::strcmp(key, "split_threshold") == 0 && value >= kTile32) {
        c->split_threshold = value;
        return PDHG_OK;
    }
    if (std::strcmp(key, "split_chunk") == 0 && value >= kWG) {
        c->split_chunk = value;
        return PDHG_OK;
    }
    const bool pv = value == 0 || value == 1 || value == 2 || value == 4 || value == 8;
    if (std::strcmp(key, "panels_a") == 0 && pv) {
        c->panels_a = (int)value;
        return PDHG_OK;
    }
    if (std::strcmp(key, "panels_at") == 0 && pv) {
        c->panels_at = (int)value;
        return PDHG_OK;
    }
    if (std::strcmp(key, "stream_nt") == 0 && value >= -1 && value <= 1) {
        c->stream_nt = (int)value;
        return PDHG_OK;
    }
    if (std::strcmp(key, "block_rows") == 0 && value >= 0 && value <= (1 << 20)) {
        c->block_rows = (int)value;
        return PDHG_OK;
    }
    if (std::strcmp(key, "sort_rows") == 0 && value >= -1 && value <= 1) {
        c->sort_rows = (int)value;
        return PDHG_OK;
    }
    if (std::strcmp(key, "sort_cols") == 0 && value >= -1 && value <= 1) {
        c->sort_cols = (int)value;
        return PDHG_OK;
    }
    return fail(c, PDHG_E_ARG, "unknown tuning key or value out of range");
}

int pdhg_load(pdhg_ctx *c, int64_t m, int64_t n, int64_t nnz,
              const int64_t *a_rp, const int32_t *a_ci, const double *a_v,
              const int64_t *at_rp, const int32_t *at_ci, const double *at_v,
              const double *b, const double *cvec, const double *lb,
              int mem) {
    API_BEGIN(c)
    if (m < 1 || n < 1 || nnz < 0 || !a_rp || !at_rp || !b || !cvec ||
        (mem != PDHG_MEM_HOST && mem != PDHG_MEM_DEVICE))
        return fail(c, PDHG_E_ARG, "bad argument to pdhg_load");
    if (nnz > 0 && (!a_ci || !a_v || !at_ci || !at_v))
        return fail(c, PDHG_E_ARG, "null CSR array");
    auto h_arp = to_host(c, a_rp, m + 1, mem);
    auto h_atrp = to_host(c, at_rp, n + 1, mem);
    auto h_aci = to_host(c, a_ci, nnz, mem);
    auto h_atci = to_host(c, at_ci, nnz, mem);
    auto h_av = to_host(c, a_v, nnz, mem);
    auto h_atv = to_host(c, at_v, nnz, mem);
    char msg[256] = {0};
    int rc = pdhg_check_transpose(m, n, nnz, h_arp.data(), h_aci.data(),
                                  h_av.data(), h_atrp.data(), h_atci.data(),
                                  h_atv.data(), nullptr, msg, sizeof msg);
    if (rc != PDHG_OK) return fail(c, rc, msg);
    std::vector<int32_t>().swap(h_atci);
    std::vector<double>().swap(h_atv);
    free_problem(c);
    c->m = m;
    c->n = n;
    c->nnz = nnz;
    // column panels: the dual step gathers x (n entries) over A's rows, the
    // primal step y (m entries) over A^T's rows
    int pa = c->panels_a ? c->panels_a : choose_panels(m, n, nnz);
    int pat = c->panels_at ? c->panels_at : choose_panels(n, m, nnz);
    // stacked panel rows are indexed in int32: keep P * rows below 2^31
    while (pa > 1 && (int64_t)pa * m >= ((int64_t)1 << 31)) pa /= 2;
    while (pat > 1 && (int64_t)pat * n >= ((int64_t)1 << 31)) pat /= 2;
    Relabeled R = relabel(m, n, nnz, h_arp.data(), h_aci.data(), h_av.data(),
                          h_atrp.data(), pa, pat, c->sort_rows, c->sort_cols);
    std::vector<int32_t>().swap(h_aci);
    std::vector<double>().swap(h_av);
    upload_csr(c, c->A, m, n, nnz, R.a_rp, R.a_ci, R.a_v, pa, R.a_cut);
    upload_csr(c, c->At, n, m, nnz, R.at_rp, R.at_ci, R.at_v, pat, R.at_cut);
    std::vector<int32_t> ridx((size_t)nnz);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = R.a_rp[i]; p < R.a_rp[i + 1]; ++p) ridx[p] = (int32_t)i;
    c->perm = dmalloc<int32_t>(nnz);
    c->rowidx = dmalloc<int32_t>(nnz);
    c->apos = dmalloc<int32_t>(nnz);
    c->pr = dmalloc<int32_t>(m);
    c->pc = dmalloc<int32_t>(n);
    if (nnz) {
        HIPC(hipMemcpy(c->perm, R.perm.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPC(hipMemcpy(c->rowidx, ridx.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPC(hipMemcpy(c->apos, R.apos.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    HIPC(hipMemcpy(c->pr, R.pr.data(), m * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(c->pc, R.pc.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
    c->tmp_m = dmalloc<double>(m);
    c->tmp_n = dmalloc<double>(n);
    c->b_orig = dmalloc<double>(m);
    c->c_orig = dmalloc<double>(n);
    vec_in(c, c->b_orig, b, true, mem);
    vec_in(c, c->c_orig, cvec, false, mem);
    c->has_l = lb != nullptr;
    if (c->has_l) {
        c->l_orig = dmalloc<double>(n);
        vec_in(c, c->l_orig, lb, false, mem);
    }
    c->dr = dmalloc<double>(m);
    c->dc = dmalloc<double>(n);
    c->bs = dmalloc<double>(m);
    c->cs = dmalloc<double>(n);
    c->ls = dmalloc<double>(n);
    c->bs32 = dmalloc<float>(m);
    c->cs32 = dmalloc<float>(n);
    c->ls32 = dmalloc<float>(n);
    c->aty_cur = dmalloc<double>(n);
    c->aty_avg = dmalloc<double>(n);
    c->ax_avg = dmalloc<double>(m);
    c->ax_cur = dmalloc<double>(m);
    c->xo = dmalloc<double>(n);
    c->yo = dmalloc<double>(m);
    c->rho = dmalloc<double>(m);
    c->kap = dmalloc<double>(n);
    c->partial = dmalloc<double>(2 * Q_NQ * 2 * kRedBlocks);
    c->scal = dmalloc<double>(16);
    c->log = dmalloc<double>(8 * (int64_t)c->log_cap);
    // until configure: unit scaling so that pdhg_spmv works on A~ = A
    launch_fill(c->dr, 1.0, m, c->stream);
    launch_fill(c->dc, 1.0, n, c->stream);
    apply_scaling(c);
    sync(c);
    c->loaded = true;
    c->configured = false;
    return PDHG_OK;
    API_END(c)
}

int pdhg_set_values(pdhg_ctx *c, const double *a_v, int mem) {
    API_BEGIN(c)
    if (!c->loaded) return fail(c, PDHG_E_STATE, "no problem loaded");
    if (!a_v && c->nnz) return fail(c, PDHG_E_ARG, "null values");
    ++c->data_gen;
    double *tmp = dmalloc<double>(c->nnz);
    copy_in(c, tmp, a_v, c->nnz, mem);
    launch_gather(c->A.v_orig, tmp, c->apos, c->nnz, c->stream);
    launch_permute(c->At.v_orig, c->A.v_orig, c->perm, c->nnz, c->stream);
    sync(c);
    dfree(tmp);
    apply_scaling(c);
    sync(c);
    return PDHG_OK;
    API_END(c)
}

int pdhg_set_rhs_obj(pdhg_ctx *c, const double *b, const double *cv, int mem) {
    API_BEGIN(c)
    if (!c->loaded) return fail(c, PDHG_E_STATE, "no problem loaded");
    if (b || cv) ++c->data_gen;
    if (b) vec_in(c, c->b_orig, b, true, mem);
    if (cv) vec_in(c, c->c_orig, cv, false, mem);
    apply_rhs_scaling(c);
    sync(c);
    return PDHG_OK;
    API_END(c)
}

}  // extern "C"

namespace {

// The start of a solve from the scaled FP64 pair (xo, yo): iterate, restart
// point, A~x and the Halpern anchor in the active precision.
void start_iterate(pdhg_ctx *c) {
    if (f32(c)) {
        zero_iter(c, c->v32);
        launch_to_f32(c->v32.x, c->xo, c->n, c->stream);
        launch_to_f32(c->v32.y, c->yo, c->m, c->stream);
        HIPC(hipMemcpyAsync(c->v32.xl, c->v32.x, c->n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
        HIPC(hipMemcpyAsync(c->v32.yl, c->v32.y, c->m * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
        spmv_f32(c->A, c->v32.x, c->v32.ax, c->stream);
        HIPC(hipMemcpyAsync(c->v32.ax0, c->v32.ax, c->m * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    } else {
        zero_iter(c, c->v64);
        HIPC(hipMemcpyAsync(c->v64.x, c->xo, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HIPC(hipMemcpyAsync(c->v64.y, c->yo, c->m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HIPC(hipMemcpyAsync(c->v64.xl, c->xo, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HIPC(hipMemcpyAsync(c->v64.yl, c->yo, c->m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        spmv_f64(c->A, c->A.v64, c->v64.x, c->v64.ax, c->stream);
        HIPC(hipMemcpyAsync(c->v64.ax0, c->v64.ax, c->m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    }
}

template <typename T>
void copy_iter(pdhg_ctx *c, Iter<T> &dst, const Iter<T> &src) {
    const size_t n = c->n * sizeof(T), m = c->m * sizeof(T);
    for (auto pr : {std::make_pair(dst.x, src.x), std::make_pair(dst.xbar, src.xbar),
                    std::make_pair(dst.xl, src.xl)})
        HIPC(hipMemcpyAsync(pr.first, pr.second, n, hipMemcpyDeviceToDevice, c->stream));
    for (auto pr : {std::make_pair(dst.y, src.y), std::make_pair(dst.ybar, src.ybar),
                    std::make_pair(dst.yl, src.yl), std::make_pair(dst.ax, src.ax),
                    std::make_pair(dst.ax0, src.ax0)})
        HIPC(hipMemcpyAsync(pr.first, pr.second, m, hipMemcpyDeviceToDevice, c->stream));
}

// One feasibility polishing attempt (see pdhg_iterate), called by the
// iteration loop after an evaluation that asked for it; the candidate waits
// unscaled in pol_x / pol_y.  The main solve (iterate, control state, host
// bookkeeping) is set aside, the two phases run as solves of their own on
// the same scaled matrix, and the main solve comes back either converged
// at the polished pair or unchanged with its next polishing point at 2k.
void polish(pdhg_ctx *c) {
    const State main_st = *c->st_host;
    const int64_t k = main_st.k, E = c->params.eval_every;
    int64_t budget = (int64_t)std::ceil(c->params.polish_frac * (double)k / (double)E) * E;
    if (budget < E) budget = E;
    const bool h = f32(c);
    if (h) {
        alloc_iter(c->bk32, c->m, c->n);
        copy_iter(c, c->bk32, c->v32);
    } else {
        alloc_iter(c->bk64, c->m, c->n);
        copy_iter(c, c->bk64, c->v64);
    }
    const pdhg_params saved = c->params;
    const std::vector<double> saved_levels = c->levels;
    const int saved_slots = c->n_slots;
    const bool saved_initial = c->initial_done, saved_keep = c->keep_snaps;
    const double saved_t_start = c->t_start, saved_t_iter = c->t_iter;
    c->keep_snaps = true;
    c->levels.clear();
    c->n_slots = 0;
    c->params.polish = 0;
    c->params.n_levels = 0;
    c->params.literal_snapshots = 0;
    c->params.max_iters = budget;
    int64_t used = 0;
    // one phase from the scaled start (xo, yo): a solve of its own that stops
    // on rel_p (mode 1) or rel_d (mode 2), logging nothing
    auto phase = [&](int mode) {
        start_iterate(c);
        State s = fresh_state(c, main_st.omega, mode == 1 ? c->nb : 0.0,
                              mode == 1 ? 0.0 : c->nc);
        s.stop_on = mode;
        s.log_cap = 0;
        write_state(c, s);
        *c->st_host = s;
        c->initial_done = false;
        c->k_host = 0;
        c->status = PDHG_RUNNING;
        run_iterations(c, budget, budget);
        used += c->k_host;
        return c->status == PDHG_CONVERGED;
    };
    // the main solve back (also when a phase throws)
    auto restore = [&]() {
        c->params = saved;
        c->levels = saved_levels;
        c->n_slots = saved_slots;
        configure_solve_state(c);
        if (h)
            copy_iter(c, c->v32, c->bk32);
        else
            copy_iter(c, c->v64, c->bk64);
        c->initial_done = saved_initial;
        c->keep_snaps = saved_keep;
        c->t_start = saved_t_start;
        c->t_iter = saved_t_iter;
    };
    bool ok = false;
    try {
        // primal phase: min 0 s.t. A~x = b~, x >= l~, from (x, 0)
        c->act_bs = c->bs;
        c->act_cs = c->zero_n;
        c->act_ls = c->ls;
        c->act_has_l = c->has_l;
        c->v64.bs = c->bs;
        c->v64.cs = c->zero_n;
        c->v64.ls = c->ls;
        c->v32.bs = c->bs32;
        c->v32.cs = c->zero_n32;
        c->v32.ls = c->ls32;
        launch_ew(c->xo, c->pol_x, c->dc, c->n, 1, c->stream);
        launch_fill(c->yo, 0.0, c->m, c->stream);
        if (phase(1)) {
            if (h)
                launch_to_f64(c->pol_xp, c->v32.x, c->n, c->stream);
            else
                HIPC(hipMemcpyAsync(c->pol_xp, c->v64.x, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            // dual phase: min c~^T x s.t. A~x = 0, x >= 0, from (0, y)
            c->act_bs = c->zero_m;
            c->act_cs = c->cs;
            c->act_ls = c->zero_n;
            c->act_has_l = false;
            c->v64.bs = c->zero_m;
            c->v64.cs = c->cs;
            c->v64.ls = c->zero_n;
            c->v32.bs = c->zero_m32;
            c->v32.cs = c->cs32;
            c->v32.ls = c->zero_n32;
            launch_fill(c->xo, 0.0, c->n, c->stream);
            launch_ew(c->yo, c->pol_y, c->dr, c->m, 1, c->stream);
            if (phase(2)) {
                if (h)
                    launch_to_f64(c->pol_yd, c->v32.y, c->m, c->stream);
                else
                    HIPC(hipMemcpyAsync(c->pol_yd, c->v64.y, c->m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
                pdhg_kkt K;
                kkt_pair64(c, c->pol_xp, c->pol_yd, c->bs, c->cs, c->has_l ? c->ls : nullptr,
                           c->nb, c->nc, &K);
                ok = K.maxresid <= saved.eps_rel;
            }
        }
    } catch (...) {
        restore();
        write_state(c, main_st);
        *c->st_host = main_st;
        throw;
    }
    restore();
    c->polish_attempts += 1;
    c->polish_iters += used;
    State s = main_st;
    s.polish_due = 0;
    if (ok) {
        // the polished pair becomes the returned iterate
        if (h) {
            launch_to_f32(c->v32.x, c->pol_xp, c->n, c->stream);
            launch_to_f32(c->v32.y, c->pol_yd, c->m, c->stream);
            spmv_f32(c->A, c->v32.x, c->v32.ax, c->stream);
        } else {
            HIPC(hipMemcpyAsync(c->v64.x, c->pol_xp, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            HIPC(hipMemcpyAsync(c->v64.y, c->pol_yd, c->m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            spmv_f64(c->A, c->A.v64, c->v64.x, c->v64.ax, c->stream);
        }
        s.status = PDHG_CONVERGED;
        s.returned_cand = 2;
        s.copy_pending = 0;
        s.snap_n = 0;
    } else {
        s.next_polish = 2 * k;
    }
    write_state(c, s);
    *c->st_host = s;
    c->status = s.status;
    c->k_host = s.k;
}

}  // namespace

extern "C" {

int pdhg_configure(pdhg_ctx *c, const pdhg_params *p) {
    API_BEGIN(c)
    if (!c->loaded) return fail(c, PDHG_E_STATE, "no problem loaded");
    if (!p) return fail(c, PDHG_E_ARG, "null params");
    if (p->eval_every < 1 || p->ruiz_passes < 0 || p->power_iters < 0 ||
        p->n_levels < 0 || p->n_levels > kMaxLevels ||
        (p->n_levels > 0 && !p->levels) ||
        (p->precision != PDHG_FP64 && p->precision != PDHG_FP32) ||
        !(p->eps_rel >= 0.0) || p->max_iters < 0 ||
        (p->variant != 0 && p->variant != 1) || !(p->reflect >= 0.0 && p->reflect <= 1.0) ||
        (p->omega_rule != 0 && p->omega_rule != 1) ||
        p->stop_on < 0 || p->stop_on > 2 || (p->polish != 0 && p->polish != 1) ||
        (p->polish && !(p->polish_frac > 0.0)))
        return fail(c, PDHG_E_ARG, "invalid parameters");
    for (int i = 1; i < p->n_levels; ++i)
        if (!(p->levels[i] < p->levels[i - 1]))
            return fail(c, PDHG_E_ARG, "snapshot levels must be strictly descending");
    const double t0 = now_s();
    invalidate_graph(c);
    ++c->data_gen;              // new scaling: earlier tapes are stale
    c->params = *p;
    c->levels.assign(p->levels, p->levels + p->n_levels);
    c->params.levels = nullptr;
    c->prec = p->precision;
    if (c->prec == PDHG_FP32)
        alloc_iter(c->v32, c->m, c->n);
    else
        alloc_iter(c->v64, c->m, c->n);
    if (c->n_slots < (int)c->levels.size()) {
        dfree(c->slots);
        c->n_slots = (int)c->levels.size();
        c->slots = dmalloc<double>((int64_t)c->n_slots * (2 * c->n + c->m));
    }
    if (p->polish && !c->pol_x) {
        c->pol_x = dmalloc<double>(c->n);
        c->pol_y = dmalloc<double>(c->m);
        c->pol_xp = dmalloc<double>(c->n);
        c->pol_yd = dmalloc<double>(c->m);
        c->zero_n = dmalloc<double>(c->n);
        c->zero_m = dmalloc<double>(c->m);
        c->zero_n32 = dmalloc<float>(c->n);
        c->zero_m32 = dmalloc<float>(c->m);
        launch_fill(c->zero_n, 0.0, c->n, c->stream);
        launch_fill(c->zero_m, 0.0, c->m, c->stream);
        launch_fill32(c->zero_n32, 0.0f, c->n, c->stream);
        launch_fill32(c->zero_m32, 0.0f, c->m, c->stream);
    }
    c->polish_attempts = 0;
    c->polish_iters = 0;
    ruiz(c, p->ruiz_passes);
    apply_scaling(c);
    apply_rhs_scaling(c);
    configure_solve_state(c);
    c->sigma_hat = 0.0;
    if (p->eta > 0.0) {
        c->eta = p->eta;
    } else {
        c->sigma_hat = power_iteration(c, p->power_iters);
        c->eta = p->eta_factor / c->sigma_hat;
    }
    const double nbs = dev_norm(c, c->bs, c->m), ncs = dev_norm(c, c->cs, c->n);
    if (p->omega0 > 0.0)
        c->omega0 = p->omega0;
    else
        c->omega0 = (nbs > 1e-10 && ncs > 1e-10) ? ncs / nbs : 1.0;
    if (c->prec == PDHG_FP32)
        zero_iter(c, c->v32);
    else
        zero_iter(c, c->v64);
    c->st_init = fresh_state(c, c->omega0, c->nb, c->nc);
    write_state(c, c->st_init);
    *c->st_host = c->st_init;
    reset_solve(c);
    c->configured = true;
    c->t_setup = now_s() - t0;
    return PDHG_OK;
    API_END(c)
}

int pdhg_set_iterate(pdhg_ctx *c, const double *x, const double *y, int mem) {
    API_BEGIN(c)
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    // scaled start in FP64 scratch: x~ = x / D_c, y~ = y / D_r
    if (x) {
        vec_in(c, c->xo, x, false, mem);
        launch_ew(c->xo, c->xo, c->dc, c->n, 1, c->stream);
    } else {
        launch_fill(c->xo, 0.0, c->n, c->stream);
    }
    if (y) {
        vec_in(c, c->yo, y, true, mem);
        launch_ew(c->yo, c->yo, c->dr, c->m, 1, c->stream);
    } else {
        launch_fill(c->yo, 0.0, c->m, c->stream);
    }
    start_iterate(c);
    c->polish_attempts = 0;
    c->polish_iters = 0;
    write_state(c, c->st_init);
    *c->st_host = c->st_init;
    reset_solve(c);
    return PDHG_OK;
    API_END(c)
}

int pdhg_iterate(pdhg_ctx *c, int64_t max_iters, int *status) {
    API_BEGIN(c)
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    if (max_iters < 0) return fail(c, PDHG_E_ARG, "negative max_iters");
    int s = run_iterations(c, max_iters, c->params.max_iters);
    if (status) *status = s;
    return PDHG_OK;
    API_END(c)
}

int pdhg_cancel(pdhg_ctx *c) {
    if (!c) return PDHG_E_ARG;
    c->cancel_flag.store(1);
    return PDHG_OK;
}

int pdhg_get_info(pdhg_ctx *c, pdhg_info *o) {
    API_BEGIN(c)
    if (!o) return fail(c, PDHG_E_ARG, "null out");
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    read_state(c);
    const State &s = *c->st_host;
    std::memset(o, 0, sizeof *o);
    o->status = c->status;
    o->candidate = s.returned_cand;
    o->iters = s.k;
    o->restarts = s.restarts;
    o->n_snap = (int)c->snaps.size();
    o->sigma_hat = c->sigma_hat;
    o->eta = c->eta;
    o->omega0 = c->omega0;
    o->omega = s.omega;
    o->tau = s.tau;
    o->sigma = s.sigma;
    o->t_setup = c->t_setup;
    o->t_iter = c->t_iter;
    o->polish_attempts = c->polish_attempts;
    o->polish_iters = c->polish_iters;
    kkt_of(c, 0, &o->kkt);
    return PDHG_OK;
    API_END(c)
}

int pdhg_residuals(pdhg_ctx *c, int which, pdhg_kkt *out) {
    API_BEGIN(c)
    if (!out || which < 0 || which > 2) return fail(c, PDHG_E_ARG, "bad argument");
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    read_state(c);
    if (which < 2) {
        kkt_of(c, which, out);
    } else {
        // the better of the two by maxresid (a tie goes to the current)
        pdhg_kkt k1;
        kkt_of(c, 0, out);
        kkt_of(c, 1, &k1);
        if (k1.maxresid < out->maxresid) *out = k1;
    }
    return PDHG_OK;
    API_END(c)
}

int pdhg_get_iterate(pdhg_ctx *c, double *x, double *y, double *z, int mem) {
    API_BEGIN(c)
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    current_products(c, false);
    double *dx = c->xo, *dy = c->yo, *dz = c->aty_avg;
    if (f32(c))
        launch_unscale_xyz32(c->v32.x, c->v32.y, c->aty_cur, c->act_cs, c->dr,
                             c->dc, c->pr, c->pc, dx, dy, dz, c->m, c->n,
                             c->stream);
    else
        launch_unscale_xyz(c->v64.x, c->v64.y, c->aty_cur, c->act_cs, c->dr,
                           c->dc, c->pr, c->pc, dx, dy, dz, c->m, c->n,
                           c->stream);
    copy_out(c, x, dx, c->n, mem);
    copy_out(c, y, dy, c->m, mem);
    copy_out(c, z, dz, c->n, mem);
    sync(c);
    return PDHG_OK;
    API_END(c)
}

int pdhg_get_scaling(pdhg_ctx *c, double *dr, double *dc, int mem) {
    API_BEGIN(c)
    if (!c->loaded) return fail(c, PDHG_E_STATE, "no problem loaded");
    vec_out(c, dr, c->dr, true, mem);
    sync(c);
    vec_out(c, dc, c->dc, false, mem);
    sync(c);
    return PDHG_OK;
    API_END(c)
}

int pdhg_eval_log(pdhg_ctx *c, double *out, int cap, int *count) {
    API_BEGIN(c)
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    read_state(c);
    const int nlog = c->st_host->n_log;
    if (count) *count = nlog;
    const int k = std::min(nlog, std::max(cap, 0));
    if (out && k > 0) {
        HIPC(hipMemcpyAsync(out, c->log, (size_t)k * 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        sync(c);
    }
    return PDHG_OK;
    API_END(c)
}

int pdhg_snapshot_count(pdhg_ctx *c, int *count) {
    if (!c || !count) return PDHG_E_ARG;
    *count = (int)c->snaps.size();
    return PDHG_OK;
}

int pdhg_snapshot(pdhg_ctx *c, int idx, pdhg_snapshot_info *info, double *x,
                  double *y, double *z, int mem) {
    API_BEGIN(c)
    if (idx < 0 || idx >= (int)c->snaps.size())
        return fail(c, PDHG_E_ARG, "snapshot index out of range");
    const SnapMeta &sm = c->snaps[idx];
    if (info) *info = sm.info;
    const double *base = c->slots + (int64_t)sm.slot * (2 * c->n + c->m);
    copy_out(c, x, base, c->n, mem);
    copy_out(c, y, base + c->n, c->m, mem);
    copy_out(c, z, base + c->n + c->m, c->n, mem);
    sync(c);
    return PDHG_OK;
    API_END(c)
}

int pdhg_set_snapshot_callback(pdhg_ctx *c, pdhg_snapshot_cb cb, void *user) {
    API_BEGIN(c)
    {
        // snapshots already queued keep the callback they were queued with
        std::lock_guard<std::mutex> lk(c->cb_mu);
        c->cb = cb;
        c->cb_user = user;
    }
    if (cb && !c->cb_thread.joinable()) {
        c->cb_stop = false;
        c->cb_thread = std::thread(cb_worker, c);
    }
    return PDHG_OK;
    API_END(c)
}

int pdhg_spmv(pdhg_ctx *c, int which, int scaled, int precision,
              const double *in, double *out, int mem) {
    API_BEGIN(c)
    if (!c->loaded) return fail(c, PDHG_E_STATE, "no problem loaded");
    if (which < 0 || which > 1 || !in || !out) return fail(c, PDHG_E_ARG, "bad argument");
    const DevCsr &M = which ? c->At : c->A;
    SpmvStage st;
    st.din = dmalloc<double>(M.cols);
    st.dout = dmalloc<double>(M.rows);
    if (precision == PDHG_FP32) {
        st.i32 = dmalloc<float>(M.cols);
        st.o32 = dmalloc<float>(M.rows);
    }
    try {
        spmv_staged(c, which, scaled, precision, in, out, mem, st);
    } catch (...) {
        (void)hipStreamSynchronize(c->stream);
        dfree(st.din), dfree(st.dout), dfree(st.i32), dfree(st.o32);
        throw;
    }
    dfree(st.din), dfree(st.dout), dfree(st.i32), dfree(st.o32);
    return PDHG_OK;
    API_END(c)
}

int pdhg_spmv_noalloc(pdhg_ctx *c, int which, int scaled, int precision,
                      const double *in, double *out, int mem) {
    API_BEGIN(c)
    if (!c->loaded) return fail(c, PDHG_E_STATE, "no problem loaded");
    if (which < 0 || which > 1 || !in || !out) return fail(c, PDHG_E_ARG, "bad argument");
    if (!c->scratch) return fail(c, PDHG_E_STATE, "no device scratch");
    const DevCsr &M = which ? c->At : c->A;
    const size_t need = spmv_noalloc_bytes(M.cols, M.rows, precision);
    if (need > kScratchBytes)
        return fail(c, PDHG_E_ARG,
                    "pdhg_spmv_noalloc: staging of " + std::to_string(need) +
                        " bytes exceeds the " + std::to_string(kScratchBytes) +
                        "-byte device scratch (rows + cols too large)");
    // carve the staging vectors out of the scratch, 256-byte aligned
    unsigned char *base = (unsigned char *)c->scratch;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = base + off;
        off += (bytes + 255) & ~(size_t)255;
        return (void *)p;
    };
    SpmvStage st;
    st.din = (double *)take((size_t)M.cols * sizeof(double));
    st.dout = (double *)take((size_t)M.rows * sizeof(double));
    if (precision == PDHG_FP32) {
        st.i32 = (float *)take((size_t)M.cols * sizeof(float));
        st.o32 = (float *)take((size_t)M.rows * sizeof(float));
    }
    spmv_staged(c, which, scaled, precision, in, out, mem, st);
    return PDHG_OK;
    API_END(c)
}

int pdhg_gather_probe(pdhg_ctx *c, int64_t table_entries, int precision,
                      int panels, int stream_nt, int64_t n_gathers, int reps,
                      double *gathers_per_s) {
    API_BEGIN(c)
    if (!gathers_per_s || table_entries < 1 || table_entries >= ((int64_t)1 << 31) ||
        (precision != PDHG_FP64 && precision != PDHG_FP32) ||
        !(panels == 1 || panels == 2 || panels == 4 || panels == 8) ||
        table_entries < panels || n_gathers < 1 || n_gathers >= ((int64_t)1 << 40) ||
        reps < 1 || reps > 1000 || stream_nt < 0 || stream_nt > 1)
        return fail(c, PDHG_E_ARG, "bad argument to pdhg_gather_probe");
    const int64_t chunk = 4096;                   // pairs per workgroup
    const int64_t npad = ((n_gathers + 3) & ~(int64_t)3) + 4;
    const int64_t nwg = (n_gathers + chunk - 1) / chunk;
    const size_t es = precision == PDHG_FP32 ? 4 : 8;
    int32_t *idx = nullptr;
    void *val = nullptr, *tab = nullptr, *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&] {
        (void)hipStreamSynchronize(c->stream);
        dfree(idx);
        if (val) (void)hipFree(val);
        if (tab) (void)hipFree(tab);
        if (out) (void)hipFree(out);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    try {
        idx = dmalloc<int32_t>(npad);
        HIPC(hipMalloc(&val, (size_t)npad * es));
        HIPC(hipMalloc(&tab, (size_t)table_entries * es));
        HIPC(hipMalloc(&out, (size_t)nwg * es));
        launch_probe_fill(idx, npad, chunk, table_entries, panels, 0x5eedull, c->stream);
        if (precision == PDHG_FP32) {
            launch_fill32((float *)val, 1.0f, npad, c->stream);
            launch_fill32((float *)tab, 0.5f, table_entries, c->stream);
        } else {
            launch_fill((double *)val, 1.0, npad, c->stream);
            launch_fill((double *)tab, 0.5, table_entries, c->stream);
        }
        auto run = [&] {
            if (precision == PDHG_FP32)
                launch_gather_probe<float>(idx, (const float *)val, (const float *)tab,
                                           chunk, n_gathers, stream_nt != 0,
                                           (float *)out, c->stream);
            else
                launch_gather_probe<double>(idx, (const double *)val, (const double *)tab,
                                            chunk, n_gathers, stream_nt != 0,
                                            (double *)out, c->stream);
        };
        run();                                    // warm-up (table into the caches)
        HIPC(hipEventCreate(&e0));
        HIPC(hipEventCreate(&e1));
        HIPC(hipEventRecord(e0, c->stream));
        for (int r = 0; r < reps; ++r) run();
        HIPC(hipEventRecord(e1, c->stream));
        HIPC(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPC(hipEventElapsedTime(&ms, e0, e1));
        *gathers_per_s = ms > 0.0f ? (double)n_gathers * reps / (ms * 1e-3) : 0.0;
    } catch (...) {
        release();
        throw;
    }
    release();
    return PDHG_OK;
    API_END(c)
}

int pdhg_bin_stats(pdhg_ctx *c, int which, int64_t *out3) {
    if (!c || !out3 || which < 0 || which > 1) return PDHG_E_ARG;
    if (!c->loaded) return fail(c, PDHG_E_STATE, "no problem loaded");
    const DevCsr &M = which ? c->At : c->A;
    for (int q = 0; q < 3; ++q) out3[q] = M.counts64[q];
    return PDHG_OK;
}

int pdhg_panel_count(pdhg_ctx *c, int which, int *panels) {
    if (!c || !panels || which < 0 || which > 1) return PDHG_E_ARG;
    if (!c->loaded) return fail(c, PDHG_E_STATE, "no problem loaded");
    *panels = (which ? c->At : c->A).P;
    return PDHG_OK;
}

int pdhg_profile(pdhg_ctx *c, int enable) {
    API_BEGIN(c)
    c->profile = enable != 0;
    return PDHG_OK;
    API_END(c)
}

int pdhg_kernel_times(pdhg_ctx *c, pdhg_kernel_time *out, int cap, int *count,
                      int reset) {
    API_BEGIN(c)
    resolve_profile(c);
    const char *names[2] = {"primal_step", "dual_step"};
    if (count) *count = 2;
    for (int k = 0; k < 2 && k < cap && out; ++k) {
        std::memset(&out[k], 0, sizeof out[k]);
        std::snprintf(out[k].name, sizeof out[k].name, "%s", names[k]);
        out[k].launches = c->prof_launch[k];
        out[k].total_ms = c->prof_ms[k];
    }
    if (reset) {
        c->prof_launch[0] = c->prof_launch[1] = 0;
        c->prof_ms[0] = c->prof_ms[1] = 0;
    }
    return PDHG_OK;
    API_END(c)
}

// ------------------------------------------------------------ Algorithm 1

}  // extern "C"

namespace {

bool refine_params_ok(const pdhg_refine_params &R);
void refine_impl(pdhg_ctx *c, const pdhg_refine_params &R, pdhg_refine_info *info,
                 bool clear_cancel = true);

// Algorithm 1 (Section 3.1) around a solve: `drive` runs it and returns the
// PDHG status; every snapshot it records (and any recorded before) launches
// `fn` on a host thread, at most max_threads at a time (0: no limit; a
// later snapshot waits for a free thread).  The first call to return 1 wins:
// the others see the cancel flag, and the solve stops at its next check.
// Without a winner, a converged solve's final iterate gets `fn` on this
// thread unless a snapshot was taken from that same iterate.
int crossover_harness(pdhg_ctx *c, pdhg_crossover_fn fn, void *user,
                      int max_threads, const std::function<int()> &drive,
                      int *winner, int *status) {
    struct Job {
        int idx;
        pdhg_snapshot_info info;
        std::vector<double> x, y, z;
    };
    // the cancel word the crossover routines poll: written and read with
    // atomic operations by the library, read as a volatile int32 by callers
    alignas(4) int32_t cancel_word = 0;
    auto cancelled = [&] { return __atomic_load_n(&cancel_word, __ATOMIC_ACQUIRE) != 0; };
    std::atomic<int> win{-2};
    JobQueue jobs(max_threads, cancelled);
    auto run_job = [&](const std::shared_ptr<Job> &jb) {
        const int ok = fn(user, jb->idx, &jb->info, jb->x.data(), jb->y.data(),
                          jb->z.data(), (const volatile int32_t *)&cancel_word);
        if (ok == 1) {
            int expected = -2;
            if (win.compare_exchange_strong(expected, jb->idx)) {
                __atomic_store_n(&cancel_word, 1, __ATOMIC_RELEASE);
                c->cancel_flag.store(1);
                jobs.notify();
            }
        }
    };
    auto fetch = [&](int idx) {
        auto jb = std::make_shared<Job>();
        jb->idx = idx;
        jb->x.resize((size_t)c->n);
        jb->y.resize((size_t)c->m);
        jb->z.resize((size_t)c->n);
        if (idx >= 0) {
            const SnapMeta &sm = c->snaps[idx];
            jb->info = sm.info;
            const double *base = c->slots + (int64_t)sm.slot * (2 * c->n + c->m);
            HIPC(hipMemcpyAsync(jb->x.data(), base, c->n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPC(hipMemcpyAsync(jb->y.data(), base + c->n, c->m * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPC(hipMemcpyAsync(jb->z.data(), base + c->n + c->m, c->n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            sync(c);
        }
        return jb;
    };
    // a snapshot is copied to the host and queued; the PDHG loop goes on
    auto queue = [&](int idx) {
        if (cancelled()) return;
        auto jb = fetch(idx);
        jobs.push([&run_job, jb] { run_job(jb); });
    };
    int st = c->status;
    // a cancel left from an earlier call is dropped here, before any
    // crossover can win; the solve `drive` runs keeps the flag as it is
    c->cancel_flag.store(0);
    try {
        for (size_t i = 0; i < c->snaps.size() && !cancelled(); ++i) queue((int)i);
        c->snap_hook = [&](int before) {
            for (int i = before; i < (int)c->snaps.size() && !cancelled(); ++i)
                queue(i);
        };
        st = drive();
        c->snap_hook = nullptr;
        if (st == PDHG_CANCELLED) {
            // a cancel from outside (pdhg_cancel) ends the crossovers too
            __atomic_store_n(&cancel_word, 1, __ATOMIC_RELEASE);
            jobs.notify();
        }
        // Algorithm 1's last line: crossover from the converged iterate on
        // this thread, unless that iterate was already handed out
        if (!cancelled() && st == PDHG_CONVERGED &&
            (c->snaps.empty() || c->snaps.back().info.iter != c->k_host)) {
            auto jb = fetch(-1);
            pdhg_get_iterate(c, jb->x.data(), jb->y.data(), jb->z.data(), PDHG_MEM_HOST);
            std::memset(&jb->info, 0, sizeof jb->info);
            jb->info.level = c->params.eps_rel;
            jb->info.iter = c->k_host;
            jb->info.t_wall = now_s() - c->t_start;
            jobs.add_external();
            run_job(jb);
            jobs.end_external();
        }
    } catch (...) {
        c->snap_hook = nullptr;
        __atomic_store_n(&cancel_word, 1, __ATOMIC_RELEASE);
        jobs.notify();
        jobs.close_and_join();
        c->cancel_flag.store(0);
        throw;
    }
    jobs.close_and_join();
    c->cancel_flag.store(0);
    if (winner) *winner = win.load();
    if (status) *status = st;
    return PDHG_OK;
}

}  // namespace

extern "C" {

int pdhg_concurrent_crossover(pdhg_ctx *c, pdhg_crossover_fn fn, void *user,
                              int max_threads, int64_t max_iters, int *winner,
                              int *status) {
    API_BEGIN(c)
    if (!fn || max_threads < 0 || max_iters < 0)
        return fail(c, PDHG_E_ARG, "bad argument to pdhg_concurrent_crossover");
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    const int64_t target = std::min<int64_t>(c->k_host + max_iters, c->params.max_iters);
    return crossover_harness(c, fn, user, max_threads, [&]() {
        run_iterations(c, target - c->k_host, target);
        return c->status;
    }, winner, status);
    API_END(c)
}

int pdhg_concurrent_crossover_refined(pdhg_ctx *c, pdhg_crossover_fn fn,
                                      void *user, int max_threads,
                                      const pdhg_refine_params *rp,
                                      int *winner, int *status,
                                      pdhg_refine_info *info) {
    API_BEGIN(c)
    if (!fn || max_threads < 0)
        return fail(c, PDHG_E_ARG, "bad argument to pdhg_concurrent_crossover_refined");
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    pdhg_refine_params R;
    if (rp)
        R = *rp;
    else
        pdhg_refine_params_default(&R);
    if (!refine_params_ok(R)) return fail(c, PDHG_E_ARG, "invalid refinement parameters");
    return crossover_harness(c, fn, user, max_threads, [&]() {
        pdhg_refine_info ri;
        refine_impl(c, R, &ri, false);
        if (info) *info = ri;
        return (int)ri.status;
    }, winner, status);
    API_END(c)
}

// ------------------------------------------------------------ refinement

}  // extern "C"

namespace {

bool refine_params_ok(const pdhg_refine_params &R) {
    return !(R.max_rounds < 0 || R.cap_log2 < 0 || R.cap_log2 > 60 ||
             (R.inner_precision != PDHG_FP32 && R.inner_precision != PDHG_FP64));
}

// The refinement driver behind pdhg_solve_refined (R already checked);
// throws DevError on device errors.  clear_cancel: drop a cancel requested
// before the call (false under the crossover harness, whose winner may have
// cancelled already).
void refine_impl(pdhg_ctx *c, const pdhg_refine_params &R, pdhg_refine_info *info,
                 bool clear_cancel) {
    const bool in64 = R.inner_precision == PDHG_FP64;
    const double *ls = c->has_l ? c->ls : nullptr;
    const double t0 = now_s();
    alloc_iter(c->v32, c->m, c->n);
    if (!c->bh) {
        c->bh = dmalloc<double>(c->m);
        c->ch = dmalloc<double>(c->n);
        c->lh = dmalloc<double>(c->n);
        c->bh32 = dmalloc<float>(c->m);
        c->ch32 = dmalloc<float>(c->n);
        c->lh32 = dmalloc<float>(c->n);
    }
    double *xo = dmalloc<double>(c->n), *yo = dmalloc<double>(c->m);
    launch_fill(xo, 0.0, c->n, c->stream);
    launch_fill(yo, 0.0, c->m, c->stream);
    if (!c->ref_bx) {
        c->ref_bx = dmalloc<double>(c->n);
        c->ref_by = dmalloc<double>(c->m);
    }
    const pdhg_params saved = c->params;
    const std::vector<double> saved_levels = c->levels;
    const int saved_slots = c->n_slots;
    double DP = 1.0, DD = 1.0;
    // primal weight at the end of round 0 or of the last round whose inner
    // solve converged, with that round's scales (a correction round cut at
    // its budget or for a stall may end with a weight far off its LP's)
    double omega_ref = 0.0, DP_ref = 1.0, DD_ref = 1.0;
    int status = PDHG_ITER_LIMIT, r = 0;
    int64_t inner_total = 0;
    pdhg_kkt K;
    std::memset(&K, 0, sizeof K);
    c->refine_log.clear();
    c->snaps.clear();
    c->keep_snaps = true;
    // a cancel is kept across the inner solves (each would clear it)
    if (clear_cancel) c->cancel_flag.store(0);
    c->keep_cancel = true;
    // snapshots of the refined iterate at the configured levels, taken
    // whenever its FP64 maxresid is measured (before every round and at the
    // end); levels crossed together share one slot
    size_t next_level = 0;
    auto snapshot_refined = [&](const pdhg_kkt &KK) {
        const int before = (int)c->snaps.size();
        int first = -1;
        while (next_level < saved_levels.size() && KK.maxresid <= saved_levels[next_level]) {
            if (first < 0) {
                first = (int)next_level;
                double *base = c->slots + (int64_t)first * (2 * c->n + c->m);
                launch_unscale_xyz(xo, yo, c->aty_cur, c->cs, c->dr, c->dc, c->pr,
                                   c->pc, base, base + c->n, base + c->n + c->m,
                                   c->m, c->n, c->stream);
            }
            SnapMeta sm;
            std::memset(&sm, 0, sizeof sm);
            sm.info.level = saved_levels[next_level];
            sm.info.iter = inner_total;
            sm.info.maxresid = KK.maxresid;
            sm.info.t_wall = now_s() - t0;
            sm.slot = first;
            c->snaps.push_back(sm);
            ++next_level;
            if (saved.literal_snapshots) break;
        }
        start_snapshot_copies(c, before);
        if (c->snap_hook && (int)c->snaps.size() > before) c->snap_hook(before);
    };
    try {
        c->levels.clear();
        c->n_slots = 0;
        c->params.eps_rel = R.inner_eps;
        c->params.max_iters = R.max_inner_iters;
        c->params.polish = 0;           // the inner solves do not polish
        c->params.stop_on = 0;
        for (r = 0;; ++r) {
            // outer FP64 KKT of (xo, yo) on the original problem
            kkt_pair64(c, xo, yo, c->bs, c->cs, c->has_l ? c->ls : nullptr, c->nb, c->nc, &K);
            if (r > 0 && !c->refine_log.empty()) {
                // close the previous round's record with the resulting KKT
                c->refine_log[c->refine_log.size() - 10 + 7] = now_s() - t0;
            }
            snapshot_refined(K);
            if (K.maxresid <= R.outer_eps) {
                status = PDHG_CONVERGED;
                break;
            }
            if (!std::isfinite(K.maxresid)) {
                status = PDHG_NUMERICAL;
                break;
            }
            if (r > R.max_rounds) break;
            if (c->cancel_flag.load()) {
                status = PDHG_CANCELLED;
                break;
            }
            // the configure time limit bounds the whole refinement
            const double left = saved.time_limit_s - (now_s() - t0);
            if (saved.time_limit_s > 0.0 && left <= 0.0) {
                status = PDHG_TIME_LIMIT;
                break;
            }
            c->params.time_limit_s = saved.time_limit_s > 0.0 ? left : 0.0;
            // ax_cur = A~ xo, aty_cur = A~^T yo from kkt_pair64
            if (r >= 1) {
                launch_refine_delta(c->bs, c->ax_cur, c->cs, c->aty_cur, xo, ls,
                                    c->dr, c->dc, c->m, c->n, c->partial,
                                    c->scal, c->stream);
                double d2[2];
                HIPC(hipMemcpyAsync(d2, c->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
                sync(c);
                const double capP = std::ldexp(DP, R.cap_log2), capD = std::ldexp(DD, R.cap_log2);
                auto pow2floor_inv = [](double d) {
                    int e = 0;
                    const double f = std::frexp(d, &e);  // d = f 2^e, f in [0.5, 1)
                    return f == 0.5 ? std::ldexp(1.0, 1 - e) : std::ldexp(1.0, -e);
                };
                const double sP = d2[0] > 0.0 ? pow2floor_inv(d2[0]) : capP;
                const double sD = d2[1] > 0.0 ? pow2floor_inv(d2[1]) : capD;
                DP = std::min(sP, capP);
                DD = std::min(sD, capD);
            }
            launch_refine_rhs(c->bs, c->ax_cur, c->cs, c->aty_cur, xo, ls, DP,
                              DD, c->bh, c->ch, c->lh, c->m, c->n, c->stream);
            launch_to_f32(c->bh32, c->bh, c->m, c->stream);
            launch_to_f32(c->ch32, c->ch, c->n, c->stream);
            launch_to_f32(c->lh32, c->lh, c->n, c->stream);
            launch_norm_unscaled(c->bh, c->dr, c->m, c->partial, c->scal, c->stream);
            const double nbh = std::sqrt(read_scalar(c, c->scal));
            launch_norm_unscaled(c->ch, c->dc, c->n, c->partial, c->scal, c->stream);
            const double nch = std::sqrt(read_scalar(c, c->scal));
            const double nbs = dev_norm(c, c->bh, c->m), ncs = dev_norm(c, c->ch, c->n);
            double om = (nbs > 1e-10 && ncs > 1e-10) ? ncs / nbs : 1.0;
            if (R.omega_carry && r >= 1 && omega_ref > 0.0)
                om = omega_ref * (DD / DD_ref) / (DP / DP_ref);
            // inner solve of the correction LP (FP32 bulk iterations unless
            // FP64 inner solves were asked for)
            c->act_bs = c->bh;
            c->act_cs = c->ch;
            c->act_ls = c->lh;
            c->act_has_l = true;
            if (in64) {
                c->prec = PDHG_FP64;
                alloc_iter(c->v64, c->m, c->n);
                c->v64.bs = c->bh;
                c->v64.cs = c->ch;
                c->v64.ls = c->lh;
                zero_iter(c, c->v64);
            } else {
                c->prec = PDHG_FP32;
                c->v32.bs = c->bh32;
                c->v32.cs = c->ch32;
                c->v32.ls = c->lh32;
                zero_iter(c, c->v32);
            }
            State s = fresh_state(c, om, nbh, nch);
            write_state(c, s);
            reset_solve(c);
            c->ref_xo = xo;
            c->ref_yo = yo;
            c->ref_DP = DP;
            c->ref_DD = DD;
            c->ref_target = std::max(R.outer_eps, R.progress * K.maxresid);
            c->ref_best = INFINITY;
            c->ref_best_k = 0;
            c->ref_cut = false;
            // the inner solve runs to its target, its inner tolerance, a
            // stall of the refined point (stall window: 0 means 65536
            // iterations, < 0 none) or its budget.  A budget or stall end
            // without any improvement of the refined point extends the same
            // solve: budget and window double, up to 16 times the budget
            c->ref_stall = R.stall_iters < 0 ? 0 : (R.stall_iters ? R.stall_iters : 65536);
            int64_t budget = R.max_inner_iters;
            for (;;) {
                run_iterations(c, budget - c->k_host, budget);
                if (c->status != PDHG_ITER_LIMIT || c->ref_best < K.maxresid ||
                    budget >= (R.max_inner_iters << 4) || c->cancel_flag.load())
                    break;
                budget *= 2;
                c->ref_stall *= 2;
                c->ref_cut = false;
                read_state(c);
                c->st_host->status = PDHG_RUNNING;
                write_state(c, *c->st_host);
                c->status = PDHG_RUNNING;
            }
            c->ref_target = -1.0;
            // round 0 solves the LP itself: its weight is PDHG's own estimate
            // for the LP however the round ended
            if (c->status == PDHG_CONVERGED || r == 0) {
                omega_ref = c->st_host->omega;
                DP_ref = DP;
                DD_ref = DD;
            }
            inner_total += c->k_host;
            pdhg_kkt ik;
            kkt_of(c, 0, &ik);
            // the round's refined point: the best its evaluations saw, or
            // the final inner iterate's when that is better; kept only if it
            // improves on the point before the round
            HIPC(hipMemcpyAsync(c->xo, xo, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            HIPC(hipMemcpyAsync(c->yo, yo, c->m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            if (in64)
                launch_refine_update<double>(c->xo, c->yo, c->v64.x, c->v64.y, ls, DP, DD, c->m, c->n, c->stream);
            else
                launch_refine_update<float>(c->xo, c->yo, c->v32.x, c->v32.y, ls, DP, DD, c->m, c->n, c->stream);
            pdhg_kkt KF;
            kkt_pair64(c, c->xo, c->yo, c->bs, c->cs, ls, c->nb, c->nc, &KF);
            const bool final_best = KF.maxresid <= c->ref_best;
            const double after = final_best ? KF.maxresid : c->ref_best;
            const bool accept = after < K.maxresid;
            if (accept) {
                const double *sx = final_best ? c->xo : c->ref_bx;
                const double *sy = final_best ? c->yo : c->ref_by;
                HIPC(hipMemcpyAsync(xo, sx, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
                HIPC(hipMemcpyAsync(yo, sy, c->m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            }
            const double rec[10] = {(double)r, K.maxresid, DP, DD,
                                    (double)c->k_host, (double)c->status,
                                    ik.maxresid, now_s() - t0,
                                    c->ref_cut ? 1.0 : 0.0, accept ? 1.0 : 0.0};
            c->refine_log.insert(c->refine_log.end(), rec, rec + 10);
            // a round that could not improve the point even with its
            // extensions would be repeated as it was: stop, reporting why the
            // inner solve ended when it was stopped from outside
            if (!accept) {
                status = c->cancel_flag.load() ? PDHG_CANCELLED
                         : c->status == PDHG_TIME_LIMIT ? PDHG_TIME_LIMIT
                         : c->status == PDHG_NUMERICAL ? PDHG_NUMERICAL
                                                       : PDHG_ITER_LIMIT;
                break;
            }
        }
    } catch (...) {
        c->ref_target = -1.0;
        c->keep_snaps = false;
        c->keep_cancel = false;
        c->params = saved;
        c->levels = saved_levels;
        c->n_slots = saved_slots;
        configure_solve_state(c);
        dfree(xo);
        dfree(yo);
        throw;
    }
    // the refined iterate becomes the current FP64 iterate
    c->params = saved;
    c->levels = saved_levels;
    c->n_slots = saved_slots;
    configure_solve_state(c);
    invalidate_graph(c);
    c->prec = PDHG_FP64;
    alloc_iter(c->v64, c->m, c->n);
    zero_iter(c, c->v64);
    HIPC(hipMemcpyAsync(c->v64.x, xo, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPC(hipMemcpyAsync(c->v64.y, yo, c->m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPC(hipMemcpyAsync(c->v64.xl, xo, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPC(hipMemcpyAsync(c->v64.yl, yo, c->m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    spmv_f64(c->A, c->A.v64, c->v64.x, c->v64.ax, c->stream);
    State s = fresh_state(c, c->omega0, c->nb, c->nc);
    s.status = status == PDHG_CONVERGED ? PDHG_CONVERGED : PDHG_RUNNING;
    s.k = inner_total;
    write_state(c, s);
    *c->st_host = s;
    c->keep_cancel = false;
    reset_solve(c);
    c->keep_snaps = false;
    c->k_host = inner_total;
    c->status = s.status;
    c->initial_done = true;
    dfree(xo);
    dfree(yo);
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->status = status;
        info->rounds = r;
        info->inner_iters = inner_total;
        info->t_total = now_s() - t0;
        info->kkt = K;
    }
}

}  // namespace

extern "C" {

int pdhg_solve_refined(pdhg_ctx *c, const pdhg_refine_params *rp,
                       pdhg_refine_info *info) {
    API_BEGIN(c)
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    pdhg_refine_params R;
    if (rp)
        R = *rp;
    else
        pdhg_refine_params_default(&R);
    if (!refine_params_ok(R)) return fail(c, PDHG_E_ARG, "invalid refinement parameters");
    refine_impl(c, R, info);
    return PDHG_OK;
    API_END(c)
}

int pdhg_refine_log(pdhg_ctx *c, double *out, int cap, int *count) {
    if (!c) return PDHG_E_ARG;
    const int k = (int)(c->refine_log.size() / 10);
    if (count) *count = k;
    if (out)
        for (int i = 0; i < k && i < cap; ++i)
            std::memcpy(out + 10 * i, c->refine_log.data() + 10 * i, 10 * sizeof(double));
    return PDHG_OK;
}

// ------------------------------------------------------------ adjoint

}  // extern "C"

namespace {

template <typename T>
void unrolled_forward_T(pdhg_ctx *c, pdhg_tape *tp, const double *x0,
                        const double *y0, double *xK, int mem) {
    const int64_t m = c->m, n = c->n;
    const int nck = tp->nseg;
    tp->ckx = dmalloc<T>((int64_t)nck * n);
    tp->cky = dmalloc<T>((int64_t)nck * m);
    tp->ckax = dmalloc<T>((int64_t)nck * m);
    Iter<T> w;
    w.x = dmalloc<T>(n);
    w.y = dmalloc<T>(m);
    w.ax = dmalloc<T>(m);
    if constexpr (sizeof(T) == 8) {
        w.bs = c->bs; w.cs = c->cs; w.ls = c->ls;
    } else {
        w.bs = c->bs32; w.cs = c->cs32; w.ls = c->ls32;
    }
    // scaled start
    if (x0) {
        vec_in(c, c->xo, x0, false, mem);
        launch_ew(c->xo, c->xo, c->dc, n, 1, c->stream);
    } else {
        launch_fill(c->xo, 0.0, n, c->stream);
    }
    if (y0) {
        vec_in(c, c->yo, y0, true, mem);
        launch_ew(c->yo, c->yo, c->dr, m, 1, c->stream);
    } else {
        launch_fill(c->yo, 0.0, m, c->stream);
    }
    if constexpr (sizeof(T) == 8) {
        HIPC(hipMemcpyAsync(w.x, c->xo, n * 8, hipMemcpyDeviceToDevice, c->stream));
        HIPC(hipMemcpyAsync(w.y, c->yo, m * 8, hipMemcpyDeviceToDevice, c->stream));
        spmv_f64(c->A, c->A.v64, w.x, w.ax, c->stream);
    } else {
        launch_to_f32(w.x, c->xo, n, c->stream);
        launch_to_f32(w.y, c->yo, m, c->stream);
        spmv_f32(c->A, w.x, w.ax, c->stream);
    }
    for (int k = 0; k < tp->K; ++k) {
        if (k % tp->ck == 0) {
            const int s = k / tp->ck;
            HIPC(hipMemcpyAsync((T *)tp->ckx + (int64_t)s * n, w.x, n * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
            HIPC(hipMemcpyAsync((T *)tp->cky + (int64_t)s * m, w.y, m * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
            HIPC(hipMemcpyAsync((T *)tp->ckax + (int64_t)s * m, w.ax, m * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
        }
        launch_primal<T>(c->At, w, c->has_l, false, tp->st, 0, c->stream);
        launch_dual<T>(c->A, w, false, tp->st, 0, c->stream);
    }
    // x_K unscaled
    double *xd = c->xo;
    if constexpr (sizeof(T) == 8)
        HIPC(hipMemcpyAsync(xd, w.x, n * 8, hipMemcpyDeviceToDevice, c->stream));
    else
        launch_to_f64(xd, w.x, n, c->stream);
    launch_ew(xd, xd, c->dc, n, 0, c->stream);
    vec_out(c, xK, xd, false, mem);
    sync(c);
    dfree(w.x);
    dfree(w.y);
    dfree(w.ax);
}

template <typename T>
void unrolled_backward_T(pdhg_tape *tp, const double *gxK, double *gc,
                         double *gb, double *gA, int mem) {
    pdhg_ctx *c = tp->ctx;
    const int64_t m = c->m, n = c->n, nnz = c->nnz;
    const int ck = tp->ck;
    T *X = dmalloc<T>((int64_t)(ck + 1) * n);
    T *Y = dmalloc<T>((int64_t)(ck + 1) * m);
    T *axw = dmalloc<T>(m);
    T *gx = dmalloc<T>(n), *gx2 = dmalloc<T>(n), *gv = dmalloc<T>(n);
    T *gy = dmalloc<T>(m), *gy2 = dmalloc<T>(m);
    T *gcs = dmalloc<T>(n), *gbs = dmalloc<T>(m), *gAs = dmalloc<T>(nnz);
    HIPC(hipMemsetAsync(gy, 0, m * sizeof(T), c->stream));
    HIPC(hipMemsetAsync(gcs, 0, n * sizeof(T), c->stream));
    HIPC(hipMemsetAsync(gbs, 0, m * sizeof(T), c->stream));
    HIPC(hipMemsetAsync(gAs, 0, nnz * sizeof(T), c->stream));
    // dL/dx~_K = D_c dL/dx_K
    vec_in(c, c->xo, gxK, false, mem);
    launch_ew(c->xo, c->xo, c->dc, n, 0, c->stream);
    if constexpr (sizeof(T) == 8)
        HIPC(hipMemcpyAsync(gx, c->xo, n * 8, hipMemcpyDeviceToDevice, c->stream));
    else
        launch_to_f32(gx, c->xo, n, c->stream);
    const T *ls = nullptr;
    if constexpr (sizeof(T) == 8) ls = c->ls; else ls = c->ls32;
    Iter<T> w;
    if constexpr (sizeof(T) == 8) {
        w.bs = c->bs; w.cs = c->cs; w.ls = c->ls;
    } else {
        w.bs = c->bs32; w.cs = c->cs32; w.ls = c->ls32;
    }
    w.ax = axw;
    for (int seg = tp->nseg - 1; seg >= 0; --seg) {
        const int s0 = seg * ck, s1 = std::min(tp->K, s0 + ck);
        HIPC(hipMemcpyAsync(X, (T *)tp->ckx + (int64_t)seg * n, n * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
        HIPC(hipMemcpyAsync(Y, (T *)tp->cky + (int64_t)seg * m, m * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
        HIPC(hipMemcpyAsync(axw, (T *)tp->ckax + (int64_t)seg * m, m * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
        for (int t = 0; t < s1 - s0; ++t) {
            T *xt = X + (int64_t)t * n, *xt1 = X + (int64_t)(t + 1) * n;
            T *yt = Y + (int64_t)t * m, *yt1 = Y + (int64_t)(t + 1) * m;
            HIPC(hipMemcpyAsync(xt1, xt, n * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
            w.x = xt1;
            w.y = yt;
            launch_primal<T>(c->At, w, c->has_l, false, tp->st, 0, c->stream);
            HIPC(hipMemcpyAsync(yt1, yt, m * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
            w.y = yt1;
            launch_dual<T>(c->A, w, false, tp->st, 0, c->stream);
        }
        for (int k = s1 - 1; k >= s0; --k) {
            const int t = k - s0;
            const T *xk = X + (int64_t)t * n, *xk1 = X + (int64_t)(t + 1) * n;
            const T *yk = Y + (int64_t)t * m;
            launch_adj_dual_bwd<T>(c->At, gy, gx, xk1, ls, c->has_l, gx2, gv,
                                   gcs, tp->tau, tp->sigma, c->stream);
            launch_adj_gA<T>(c->A, c->rowidx, yk, gy, gv, xk, xk1, gAs,
                             tp->tau, tp->sigma, c->stream);
            launch_adj_primal_bwd<T>(c->A, gv, gy, gy2, gbs, tp->tau,
                                     tp->sigma, c->stream);
            std::swap(gx, gx2);
            std::swap(gy, gy2);
        }
    }
    // unscale: dL/dc = D_c dL/dc~, dL/db = D_r dL/db~,
    // dL/dA_ij = (D_r,i dL/dA~_ij) D_c,j
    double *g64 = dmalloc<double>(nnz > n ? (nnz > m ? nnz : m) : (n > m ? n : m));
    double *out = dmalloc<double>(nnz > n ? (nnz > m ? nnz : m) : (n > m ? n : m));
    auto widen = [&](const T *src, int64_t k) {
        if constexpr (sizeof(T) == 8)
            HIPC(hipMemcpyAsync(g64, src, k * 8, hipMemcpyDeviceToDevice, c->stream));
        else
            launch_to_f64(g64, src, k, c->stream);
    };
    widen(gcs, n);
    launch_ew(out, g64, c->dc, n, 0, c->stream);
    vec_out(c, gc, out, false, mem);
    sync(c);
    widen(gbs, m);
    launch_ew(out, g64, c->dr, m, 0, c->stream);
    vec_out(c, gb, out, true, mem);
    sync(c);
    widen(gAs, nnz);
    launch_scale_values(c->A, g64, c->dr, c->dc, out, nullptr, c->stream);
    launch_permute(g64, out, c->apos, nnz, c->stream);   // A's original order
    copy_out(c, gA, g64, nnz, mem);
    sync(c);
    dfree(g64);
    dfree(out);
    dfree(X);
    dfree(Y);
    dfree(axw);
    dfree(gx);
    dfree(gx2);
    dfree(gv);
    dfree(gy);
    dfree(gy2);
    dfree(gcs);
    dfree(gbs);
    dfree(gAs);
}

}  // namespace

extern "C" {

int pdhg_unrolled_forward(pdhg_ctx *c, int K, int ckpt_every, int precision,
                          double tau, double sigma, const double *x0,
                          const double *y0, double *xK, int mem,
                          pdhg_tape **tape) {
    API_BEGIN(c)
    if (!tape || !xK || K < 1 || ckpt_every < 1 || !(tau > 0.0) || !(sigma > 0.0) ||
        (precision != PDHG_FP64 && precision != PDHG_FP32))
        return fail(c, PDHG_E_ARG, "bad argument to pdhg_unrolled_forward");
    if (!c->configured) return fail(c, PDHG_E_STATE, "configure first");
    *tape = nullptr;
    pdhg_tape *tp = new pdhg_tape();
    tp->ctx = c;
    tp->data_gen = c->data_gen;
    tp->K = K;
    tp->ck = std::min(ckpt_every, K);
    tp->prec = precision;
    tp->nseg = (K + tp->ck - 1) / tp->ck;
    tp->tau = tau;
    tp->sigma = sigma;
    try {
        tp->st = dmalloc<State>(1);
        State s;
        std::memset(&s, 0, sizeof s);
        s.tau = tau;
        s.sigma = sigma;
        s.status = PDHG_RUNNING;
        HIPC(hipMemcpyAsync(tp->st, &s, sizeof s, hipMemcpyHostToDevice, c->stream));
        if (precision == PDHG_FP32)
            unrolled_forward_T<float>(c, tp, x0, y0, xK, mem);
        else
            unrolled_forward_T<double>(c, tp, x0, y0, xK, mem);
    } catch (...) {
        pdhg_tape_free(tp);
        throw;
    }
    c->tapes.push_back(tp);
    *tape = tp;
    return PDHG_OK;
    API_END(c)
}

int pdhg_unrolled_backward(pdhg_tape *tp, const double *gxK, double *gc,
                           double *gb, double *gAval, int mem) {
    if (!tp) return PDHG_E_ARG;
    if (!tp->ctx) return PDHG_E_STATE;      // its context was destroyed
    pdhg_ctx *c = tp->ctx;
    API_BEGIN(c)
    if (!gxK || !gc || !gb || !gAval) return fail(c, PDHG_E_ARG, "null argument");
    if (tp->data_gen != c->data_gen || !tp->ckx)
        return fail(c, PDHG_E_STATE,
                    "the problem data changed since this tape's forward pass "
                    "(load, configure, set_values or set_rhs_obj); run the "
                    "forward pass again");
    if (tp->prec == PDHG_FP32)
        unrolled_backward_T<float>(tp, gxK, gc, gb, gAval, mem);
    else
        unrolled_backward_T<double>(tp, gxK, gc, gb, gAval, mem);
    return PDHG_OK;
    API_END(c)
}

static void tape_release(pdhg_tape *tp) {
    if (tp->ctx) {
        (void)hipSetDevice(tp->ctx->device);
        if (tp->ctx->stream) (void)hipStreamSynchronize(tp->ctx->stream);
    }
    if (tp->ckx) (void)hipFree(tp->ckx);
    if (tp->cky) (void)hipFree(tp->cky);
    if (tp->ckax) (void)hipFree(tp->ckax);
    if (tp->st) (void)hipFree(tp->st);
    tp->ckx = tp->cky = tp->ckax = nullptr;
    tp->st = nullptr;
}

void pdhg_tape_free(pdhg_tape *tp) {
    if (!tp) return;
    if (tp->ctx) {
        auto &v = tp->ctx->tapes;
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i] == tp) {
                v.erase(v.begin() + (long)i);
                break;
            }
    }
    tape_release(tp);
    delete tp;
}

}  // extern "C"
