// smash.hip -- host side of libsmash: contexts, workspace layout, planning,
// launches and the C ABI declared in include/smash.h.
//
// Call structure (SMASH Kernels chapter: window distribution, hashing and
// write-back phases, each closed by a barrier; here every phase is a set of
// kernels ordered on the caller's stream):
//   symbolic: validate -> analyze (products per row, bins) -> bin offsets ->
//             scatter rows by bin -> per-bin LDS hash kernels (persistent,
//             bin sizes read on the device) + heavy-row kernels -> row-pointer
//             scan -> numeric bins and heavy-row segments -> [read the plan
//             header and nnz(C) back: the call's one host synchronisation]
//   numeric:  per-bin LDS hash kernels (hash, compact, sort, write) +
//             heavy-row kernels, sized from the plan header; no
//             synchronisation (device-detected errors are reported by
//             smash_sync or the next symbolic call)
// Every device buffer of a call is the caller's: inputs, outputs and one
// workspace, laid out here (plan arrays of fixed size, then the heavy-row
// tables sized from what is left).  A check that fails on the device (an
// invalid matrix, a workspace too small) sets a flag that every later kernel
// of the pipeline tests on entry, so nothing indexes through bad data, and
// the host reports it at the synchronisation.
#include "smash.h"
#include "smash_kernels.hpp"
#include "smash_mlp.hpp"
#include "smash_fused.hpp"
#include "smash_batch.hpp"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

using namespace smash;

// Workspace of smash_spgemm_noalloc: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends).  In host code
// `scratch` names a host-side stand-in, not device memory: its device address
// is resolved once per device with hipGetSymbolAddress (in smash_create, with
// the device current) and only that address is ever passed to kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace {

enum KernelId {
    K_VALIDATE, K_ANALYZE, K_BIN_COUNT, K_BIN_SCAN, K_SCATTER, K_SYM_ROWS, K_BSPLIT, K_SYM_HEAVY,
    K_SYM_GLOBAL, K_FILL, K_SCAN_REDUCE, K_SCAN_TOP, K_SCAN_APPLY, K_NUM_BINS, K_CHUNK_PREFIX,
    K_SEG_PLAN, K_SEG_SCAN, K_NUM_ROWS, K_NUM_SEG, K_NUM_DENSE, K_NUM_GLOBAL, K_FEATURES, K_MLP_PREDICT,
    K_MLP_FWD, K_MLP_BWD, K_ADAM, K_FUSED_ROWS, K_FUSED_AUX, K_FUSED_COPY, K_WS_QUERY, K_COUNT
};

const char *const kKernelNames[K_COUNT] = {
    "validate", "analyze", "bin_count", "bin_scan", "scatter", "sym_rows", "bsplit", "sym_heavy",
    "sym_global", "fill", "scan_reduce", "scan_top", "scan_apply", "num_bins", "chunk_prefix",
    "seg_plan", "seg_scan", "num_rows", "num_seg", "num_dense", "num_global", "features", "mlp_predict",
    "mlp_fwd", "mlp_bwd", "adam", "fused_rows", "fused_aux", "fused_copy", "ws_query"};

// Grow-only device buffer of the context (predictor weights, training
// buffers): not used by the multiply's calls.
struct Arena {
    void *ptr = nullptr;
    size_t cap = 0;
};

// Carves 256-byte aligned arrays out of a buffer; with base == nullptr it
// only measures (off is the bytes used so far).
struct Carve {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

size_t carve_size(std::initializer_list<size_t> parts)
{
    size_t s = 0;
    for (size_t p : parts) s += ((p + 255) & ~size_t(255)) + 256;
    return s;
}

// Bytes of the workspace per heavy row (LDS mode: chunk counts, chunk
// offsets and up to one segment per chunk) and per global hash slot (global
// mode: key, FP64 value, touched-slot list entry).
constexpr size_t kGlobalSlotBytes = sizeof(int) + sizeof(double) + sizeof(int);
constexpr size_t kCarveSlack = 4 * 256;

struct Plan {
    bool valid = false;
    smash_csr A{}, B{};
    const int64_t *crp = nullptr;
    int64_t m = 0, n = 0;
    int heavy_mode = 0, lds_row_max = 0, row_hash = 0;
    DevHdr hdr{};
    int nchunks = 0, nblk = 0;
    // workspace
    const void *ws = nullptr;
    size_t ws_bytes = 0, ws_fixed = 0;
    long long hcap = 0;                   // heavy rows the workspace holds (LDS mode)
    long long pool_cap = 0;               // global hash slots the workspace holds (global mode)
    long long *ub = nullptr;
    int *cap = nullptr, *nnzc = nullptr, *sym_perm = nullptr, *num_perm = nullptr;
    unsigned char *sym_bin = nullptr, *num_bin = nullptr;
    int *bcount = nullptr;
    unsigned long long *bprod = nullptr;
    long long *bw = nullptr;
    long long *bsum = nullptr, *gsz = nullptr, *goff_sym = nullptr, *goff_num = nullptr;
    unsigned *valid_bm = nullptr;
    int *bsplit = nullptr, *wcnt = nullptr, *woff = nullptr, *seg_bcount = nullptr;
    Seg *segs = nullptr;
    int *queue = nullptr;                 // work-queue counter of the persistent dense kernel
    int *gkeys = nullptr, *gtouch = nullptr;
    double *gvals = nullptr;
    // global mode: waves of heavy rows (first row and table offset of each
    // wave, then the end) and the pool each pass needs
    std::vector<std::pair<int, long long>> sym_waves, num_waves;
    long long sym_pool = 0, num_pool = 0;
    // fused pass (rows sized by the predictor)
    bool fused = false;
    int fused_dtype = 0;
    float *feats = nullptr;
    int *maxb = nullptr, *cap_pred = nullptr, *fcap = nullptr, *f_perm = nullptr;
    unsigned char *fbin = nullptr, *fstatus = nullptr;
    long long *stage_off = nullptr;
    long long stage_cap = 0;
    int *stage_col = nullptr;
    void *stage_val = nullptr;
};

struct Pending {
    int kid;
    hipEvent_t a, b;
};

}  // namespace

// The context's device header and the numeric error word after it, in one
// allocation (and one pinned host mirror), so one copy reads both.
constexpr size_t kNumErrOffset = (sizeof(DevHdr) + 15) & ~size_t(15);
constexpr size_t kHdrBytes = kNumErrOffset + 16;

struct smash_ctx_s {
    int device = 0;
    std::string err;
    int64_t opt[SMASH_OPT_COUNT] = {1, 1024, 0, 0, 0, 0, 0};
    DevHdr *h_hdr = nullptr;   // pinned host mirror
    DevHdr *d_hdr = nullptr;
    int *d_numerr = nullptr;   // flags of numeric calls (kept until smash_sync or a symbolic call reads them);
                               // right after the header, so one copy reads both
    int *h_numerr = nullptr;   // pinned host mirror, likewise after h_hdr
    Arena mlp_mem, pred_mem;
    bool has_predictor = false;
    float pred_delta = 0.f;
    Plan plan;
    smash_stats stats{};
    std::vector<hipEvent_t> event_pool;
    std::vector<Pending> pending;
    int64_t launches[K_COUNT] = {};
    double ms[K_COUNT] = {};
    int cus = 256;                 // compute units of the device
    void *scratch = nullptr;       // device address of `scratch` on this context's device
};

namespace {

smash_status fail(smash_ctx c, smash_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = std::string(smash_status_string(s)) + ": " + buf;
    return s;
}

#define HIP_TRY(c, call)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((c), SMASH_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

#define TRY(...)                           \
    do {                                   \
        smash_status s_ = (__VA_ARGS__);   \
        if (s_ != SMASH_OK) return s_;     \
    } while (0)

// Makes the context's device current for the scope of one call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Context-owned buffers (predictor weights and training only).
smash_status ensure(smash_ctx c, Arena &a, size_t bytes, hipStream_t s)
{
    bytes = std::max<size_t>(bytes, 256);
    if (a.cap >= bytes) return SMASH_OK;
    if (a.ptr) {
        HIP_TRY(c, hipStreamSynchronize(s));
        HIP_TRY(c, hipFree(a.ptr));
        a.ptr = nullptr;
    }
    size_t want = std::max(bytes, a.cap + a.cap / 2);
    a.cap = 0;
    if (hipMalloc(&a.ptr, want) != hipSuccess) {
        (void)hipGetLastError();
        if (hipMalloc(&a.ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            a.ptr = nullptr;
            return fail(c, SMASH_ERR_OUT_OF_MEMORY, "device allocation of %zu bytes failed", bytes);
        }
        want = bytes;
    }
    a.cap = want;
    return SMASH_OK;
}

hipEvent_t take_event(smash_ctx c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Blocks of `kernel` (block size `threads`, `lds` bytes of dynamic LDS)
// resident on the whole device at once: the grid of a persistent kernel.
int resident_blocks(smash_ctx c, const void *kernel, int threads, size_t lds)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    return per_cu * c->cus;
}

// Launches `fn` (a lambda issuing one kernel) and, with timing on, brackets
// it with events on the same stream.
template <typename F>
smash_status launch(smash_ctx c, int kid, hipStream_t s, F fn)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (c->opt[SMASH_OPT_TIMING]) {
        a = take_event(c);
        b = take_event(c);
        if (a && b) HIP_TRY(c, hipEventRecord(a, s));
    }
    fn();
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, SMASH_ERR_HIP, "launch of %s failed: %s", kKernelNames[kid], hipGetErrorString(e));
    if (a && b) {
        HIP_TRY(c, hipEventRecord(b, s));
        c->pending.push_back({kid, a, b});
    }
    return SMASH_OK;
}

// Folds timing events into the per-kernel totals (waits for the last one).
void collect_times(smash_ctx c)
{
    if (!c->pending.empty()) (void)hipEventSynchronize(c->pending.back().b);
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->ms[p.kid] += ms;
            c->launches[p.kid] += 1;
        }
        c->event_pool.push_back(p.a);
        c->event_pool.push_back(p.b);
    }
    c->pending.clear();
}

smash_status check_csr(smash_ctx c, const smash_csr *M, const char *name, bool need_val)
{
    if (!M) return fail(c, SMASH_ERR_INVALID_ARG, "%s is NULL", name);
    if (M->rows < 0 || M->cols < 0 || M->nnz < 0)
        return fail(c, SMASH_ERR_INVALID_ARG, "%s has a negative size", name);
    if (M->rows >= INT32_MAX || M->cols >= INT32_MAX || M->nnz >= INT32_MAX)
        return fail(c, SMASH_ERR_INDEX_OVERFLOW, "%s exceeds int32 indexing", name);
    if (!M->row_ptr) return fail(c, SMASH_ERR_INVALID_ARG, "%s.row_ptr is NULL", name);
    if (M->nnz > 0 && !M->col_idx) return fail(c, SMASH_ERR_INVALID_ARG, "%s.col_idx is NULL", name);
    if (need_val && M->nnz > 0 && !M->val) return fail(c, SMASH_ERR_INVALID_ARG, "%s.val is NULL", name);
    return SMASH_OK;
}

bool same_csr(const smash_csr &x, const smash_csr &y)
{
    return x.rows == y.rows && x.cols == y.cols && x.nnz == y.nnz && x.row_ptr == y.row_ptr && x.col_idx == y.col_idx;
}

unsigned blocks_for(long long items, int per_block)
{
    return (unsigned)((items + per_block - 1) / per_block);
}

int *perr(smash_ctx c) { return &c->d_hdr->error; }

// ---------------------------------------------------------- workspace layout

// Carves the fixed part of a product's workspace (per-row plan arrays,
// binning scratch, validation bitmap, the fused pass's per-row arrays, the
// split table of heavy rows) and then, from what is left of ws_bytes, the
// heavy-row tables: p.hcap heavy rows in LDS mode, p.pool_cap global slots
// in global mode.  With base == nullptr it only measures (p.ws_fixed).
void carve_workspace(smash_ctx c, Plan &p, char *base, size_t ws_bytes)
{
    const long long m = p.m;
    const bool global = p.heavy_mode == 1;
    Carve cv{base};
    p.ub = cv.take<long long>(m);
    p.cap = cv.take<int>(m);
    p.nnzc = cv.take<int>(m);
    p.sym_perm = cv.take<int>(m);
    p.num_perm = cv.take<int>(m);
    p.sym_bin = cv.take<unsigned char>(m);
    p.num_bin = cv.take<unsigned char>(m);
    p.nblk = (int)blocks_for(std::max<long long>(m, 1), kBinBlockRows);
    const int nsb = (int)blocks_for(std::max<long long>(m, 1), kScanItems);
    p.bcount = cv.take<int>((size_t)p.nblk * kNumBins);
    p.bprod = cv.take<unsigned long long>(p.nblk);
    p.bw = cv.take<long long>((size_t)p.nblk * kNumBins);
    p.bsum = cv.take<long long>((size_t)nsb + 1);
    p.queue = cv.take<int>(64);
    if (c->opt[SMASH_OPT_VALIDATE])
        p.valid_bm = cv.take<unsigned>((size_t)(std::max(p.A.nnz, p.B.nnz) + 31) / 32 + 1);
    if (p.fused) {
        p.feats = cv.take<float>((size_t)m * kFeat);
        p.maxb = cv.take<int>(m);
        p.cap_pred = cv.take<int>(m);
        p.fcap = cv.take<int>(m);
        p.f_perm = cv.take<int>(m);
        p.fbin = cv.take<unsigned char>(m);
        p.fstatus = cv.take<unsigned char>(m);
        p.stage_off = cv.take<long long>((size_t)m + 1);
    }
    if (global) {
        p.gsz = cv.take<long long>(m);
        p.goff_sym = cv.take<long long>((size_t)m + 1);
        p.goff_num = cv.take<long long>((size_t)m + 1);
    } else {
        p.bsplit = cv.take<int>((size_t)p.B.rows * (p.nchunks + 1));
        p.seg_bcount = cv.take<int>((size_t)kSegBins * p.nchunks);
    }
    p.ws_fixed = cv.off + kCarveSlack;
    const size_t rest = ws_bytes > p.ws_fixed ? ws_bytes - p.ws_fixed : 0;
    p.hcap = 0;
    p.pool_cap = 0;
    if (global) {
        p.pool_cap = (long long)(rest / kGlobalSlotBytes);
        p.gkeys = cv.take<int>(p.pool_cap);
        p.gvals = cv.take<double>(p.pool_cap);
        p.gtouch = cv.take<int>(p.pool_cap);
    } else {
        // a heavy row needs more than lds_row_max output columns: with B no
        // wider than that there are none, and no heavy-row kernel is launched
        const size_t per_row = (size_t)p.nchunks * (2 * sizeof(int) + sizeof(Seg));
        p.hcap = p.n > p.lds_row_max ? std::min<long long>((long long)(rest / per_row), m) : 0;
        const size_t cells = (size_t)p.hcap * p.nchunks;
        p.wcnt = cv.take<int>(cells);
        p.woff = cv.take<int>(cells);
        p.segs = cv.take<Seg>(cells);
    }
}

// Workspace bytes for `heavy` heavy rows (LDS mode) or `slots` global slots.
size_t workspace_need(const Plan &p, long long heavy, long long slots)
{
    if (p.heavy_mode == 1) return p.ws_fixed + (size_t)slots * kGlobalSlotBytes;
    return p.ws_fixed + (size_t)heavy * p.nchunks * (2 * sizeof(int) + sizeof(Seg));
}

// ------------------------------------------------------------- LDS bins

template <int LOGT>
struct BinShape {
    // up to 512 slots: a wave per row, four rows per block; 1024 slots: two
    // waves; 2048 slots: four waves
    static constexpr int WPR = LOGT <= 9 ? 1 : (1 << (LOGT - 9));
    static constexpr int RPW = WPR == 1 ? 4 : 1;
    static constexpr int THREADS = kWave * WPR * RPW;
};

// Persistent grid of a light-row kernel: the resident blocks, at most enough
// for every row of A.
template <typename K>
unsigned persistent_grid(smash_ctx c, K kernel, int threads, int rpw, long long m)
{
    const int res = resident_blocks(c, (const void *)kernel, threads, 0);
    return (unsigned)std::max<long long>(1, std::min<long long>(res, blocks_for(m, rpw)));
}

template <int LOGT>
smash_status launch_sym_bin(smash_ctx c, hipStream_t s, const Plan &p)
{
    using S = BinShape<LOGT>;
    auto kern = k_sym_rows<LOGT, S::WPR, S::RPW>;
    const unsigned grid = persistent_grid(c, kern, S::THREADS, S::RPW, p.m);
    return launch(c, K_SYM_ROWS, s, [&] {
        kern<<<grid, S::THREADS, 0, s>>>(p.A.row_ptr, p.A.col_idx, p.B.row_ptr, p.B.col_idx, p.sym_perm,
                                         &c->d_hdr->sym, LOGT - kMinLogT, p.nnzc, perr(c));
    });
}

template <typename V, int LOGT>
smash_status launch_num_bin(smash_ctx c, hipStream_t s, const Plan &p, int cnt, const int *rows, const V *Aval,
                            const V *Bval, const int64_t *crp, int32_t *ccol, V *cval)
{
    using S = BinShape<LOGT>;
    return launch(c, K_NUM_ROWS, s, [&] {
        if (p.row_hash)
            k_num_rows<V, LOGT, S::WPR, S::RPW, 1><<<blocks_for(cnt, S::RPW), S::THREADS, 0, s>>>(
                p.A.row_ptr, p.A.col_idx, Aval, p.B.row_ptr, p.B.col_idx, Bval, rows, cnt, (const long long *)crp,
                ccol, cval, (int)p.n, c->d_numerr);
        else
            k_num_rows<V, LOGT, S::WPR, S::RPW, 0><<<blocks_for(cnt, S::RPW), S::THREADS, 0, s>>>(
                p.A.row_ptr, p.A.col_idx, Aval, p.B.row_ptr, p.B.col_idx, Bval, rows, cnt, (const long long *)crp,
                ccol, cval, (int)p.n, c->d_numerr);
    });
}

// Symbolic light rows: every bin is launched (its size is on the device).
smash_status run_sym_bins(smash_ctx c, hipStream_t s, const Plan &p)
{
    TRY(launch_sym_bin<6>(c, s, p));
    TRY(launch_sym_bin<7>(c, s, p));
    TRY(launch_sym_bin<8>(c, s, p));
    TRY(launch_sym_bin<9>(c, s, p));
    TRY(launch_sym_bin<10>(c, s, p));
    TRY(launch_sym_bin<11>(c, s, p));
    return SMASH_OK;
}

template <typename V>
smash_status run_num_bins(smash_ctx c, hipStream_t s, const Plan &p, const V *Aval, const V *Bval,
                          const int64_t *crp, int32_t *ccol, V *cval)
{
    const BinHdr &b = p.hdr.num;
    const int *perm = p.num_perm;
#define NUM_BIN(LT)                                                                                   \
    if (b.count[LT - kMinLogT])                                                                       \
        TRY(launch_num_bin<V, LT>(c, s, p, b.count[LT - kMinLogT], perm + b.offset[LT - kMinLogT], Aval, Bval, crp, \
                                  ccol, cval));
    NUM_BIN(6) NUM_BIN(7) NUM_BIN(8) NUM_BIN(9) NUM_BIN(10) NUM_BIN(11)
#undef NUM_BIN
    return SMASH_OK;
}

// Binning of the rows by `bin_of` into `perm` (block histograms, one scan
// block, scatter), with the global-hash table sizes of heavy rows when
// gsize_of is given; heavy_cap >= 0 limits the heavy rows (workspace).
smash_status bin_rows(smash_ctx c, hipStream_t s, const Plan &p, const unsigned char *bin_of, const long long *ub,
                      const int *wt, BinHdr *dh, int *perm, const int *gsize_of, long long heavy_cap)
{
    const int m = (int)p.m;
    TRY(launch(c, K_BIN_COUNT, s, [&] {
        k_bin_count<<<p.nblk, 256, 0, s>>>(m, bin_of, ub, wt, p.bcount, ub ? p.bprod : nullptr, wt ? p.bw : nullptr,
                                           perr(c));
    }));
    TRY(launch(c, K_BIN_SCAN, s, [&] {
        k_bin_scan<<<1, 256, 0, s>>>(p.nblk, p.bcount, ub ? p.bprod : nullptr, wt ? p.bw : nullptr, dh,
                                     ub ? &c->d_hdr->products : nullptr, perr(c), heavy_cap);
    }));
    TRY(launch(c, K_SCATTER, s, [&] {
        k_scatter<<<p.nblk, 256, 0, s>>>(m, bin_of, p.bcount, dh, perm, gsize_of, p.gsz, perr(c));
    }));
    return SMASH_OK;
}

// out[0..n] = exclusive prefix of cnt[0..n) (int or int64), total in *total.
template <typename TIn>
smash_status scan_counts(smash_ctx c, hipStream_t s, long long n, const TIn *cnt, long long *bsum,
                         long long *out, long long *total)
{
    const int nb = (int)blocks_for(std::max<long long>(n, 1), kScanItems);
    TRY(launch(c, K_SCAN_REDUCE, s, [&] { k_scan_reduce<TIn><<<nb, kScanThreads, 0, s>>>(n, cnt, bsum); }));
    TRY(launch(c, K_SCAN_TOP, s, [&] { k_scan_top<<<1, kScanThreads, 0, s>>>(nb, bsum, total); }));
    TRY(launch(c, K_SCAN_APPLY, s, [&] { k_scan_apply<TIn><<<nb, kScanThreads, 0, s>>>(n, cnt, bsum, total, out); }));
    return SMASH_OK;
}

template <typename V, int LOGT, int THREADS>
smash_status launch_seg_bin(smash_ctx c, hipStream_t s, const Plan &p, int bin, const V *Aval, const V *Bval,
                            const int64_t *crp, int32_t *ccol, V *cval)
{
    const int cnt = p.hdr.seg.count[bin];
    if (!cnt) return SMASH_OK;
    const int *hrows = p.sym_perm + p.hdr.sym.offset[kBinHeavy];
    const Seg *segs = p.segs + p.hdr.seg.offset[bin];
    return launch(c, K_NUM_SEG, s, [&] {
        k_num_seg<V, LOGT, THREADS><<<cnt, THREADS, 0, s>>>(p.A.row_ptr, p.A.col_idx, Aval, p.B.col_idx, Bval, p.bsplit, (long long)(p.nchunks + 1),
                                                     hrows, segs, p.nchunks, p.woff, (const long long *)crp, ccol,
                                                     cval, c->d_numerr);
    });
}

template <typename V>
smash_status numeric_impl(smash_ctx c, hipStream_t s, const Plan &p, const V *Aval, const V *Bval,
                          const int64_t *crp, int32_t *ccol, V *cval)
{
    TRY(run_num_bins<V>(c, s, p, Aval, Bval, crp, ccol, cval));
    const int H = p.hdr.sym.count[kBinHeavy];
    if (H == 0) return SMASH_OK;
    if (p.heavy_mode == 0) {
        // segments of up to 128 entries (table of 256 slots): one wave; up to
        // 700 (1024 slots) and up to 1024 entries (2048 slots): four waves
        TRY(launch_seg_bin<V, 8, 64>(c, s, p, 0, Aval, Bval, crp, ccol, cval));
        TRY(launch_seg_bin<V, 10, 256>(c, s, p, 1, Aval, Bval, crp, ccol, cval));
        TRY(launch_seg_bin<V, 11, 256>(c, s, p, 2, Aval, Bval, crp, ccol, cval));
        const int nd = p.hdr.seg.count[kSegDense];
        if (nd) {
            const size_t lds = (size_t)kChunkCols * sizeof(double);
            (void)hipFuncSetAttribute((const void *)k_num_dense<V>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            const int *hrows = p.sym_perm + p.hdr.sym.offset[kBinHeavy];
            const Seg *segs = p.segs + p.hdr.seg.offset[kSegDense];
            // persistent: as many blocks as are resident at once, fed by a queue
            const int grid = std::min(nd, resident_blocks(c, (const void *)k_num_dense<V>, kDenseThreads, lds));
            TRY(launch(c, K_FILL, s, [&] { k_fill_i32<<<1, kWave, 0, s>>>(1, p.queue, 0); }));
            TRY(launch(c, K_NUM_DENSE, s, [&] {
                k_num_dense<V><<<grid, kDenseThreads, lds, s>>>(p.A.row_ptr, p.A.col_idx, Aval, p.B.col_idx, Bval,
                                                               p.bsplit, (long long)(p.nchunks + 1), hrows, segs, p.nchunks,
                                                               p.woff, (const long long *)crp, ccol, cval,
                                                               c->d_numerr, nd, p.queue,
                                                               nd >= kDenseClaimMinPerBlock * grid ? kDenseClaim : 1);
            }));
        }
        return SMASH_OK;
    }
    // global-memory hash tables in the workspace's pool, in the waves planned
    // by the symbolic phase (each row clears its own table, so the pool is
    // reused as it is)
    const size_t lds = (size_t)kGlobalRankBits / 8;
    (void)hipFuncSetAttribute((const void *)k_num_global<V>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int *rows = p.num_perm + p.hdr.num.offset[kBinHeavy];
    for (size_t w = 0; w + 1 < p.num_waves.size(); ++w) {
        const int h0 = p.num_waves[w].first, nh = p.num_waves[w + 1].first - h0;
        const long long base = p.num_waves[w].second;
        TRY(launch(c, K_NUM_GLOBAL, s, [&] {
            k_num_global<V><<<nh, kGlobalThreads, lds, s>>>(p.A.row_ptr, p.A.col_idx, Aval, p.B.row_ptr, p.B.col_idx,
                                                            Bval, rows + h0, (int)p.n, p.goff_num + h0, base, p.gkeys,
                                                            p.gvals, p.gtouch, (const long long *)crp, ccol, cval,
                                                            c->d_numerr);
        }));
    }
    return SMASH_OK;
}

template <typename V, int LOGT>
smash_status launch_fused_bin(smash_ctx c, hipStream_t s, const Plan &p)
{
    using S = BinShape<LOGT>;
    auto kern = k_fused_rows<V, LOGT, S::WPR, S::RPW>;
    const unsigned grid = persistent_grid(c, kern, S::THREADS, S::RPW, p.m);
    return launch(c, K_FUSED_ROWS, s, [&] {
        kern<<<grid, S::THREADS, 0, s>>>(p.A.row_ptr, p.A.col_idx, (const V *)p.A.val, p.B.row_ptr, p.B.col_idx,
                                         (const V *)p.B.val, p.f_perm, &c->d_hdr->fz, LOGT - kMinLogT, p.fcap,
                                         p.stage_off, p.stage_cap, p.stage_col, (V *)p.stage_val, p.nnzc, p.fstatus,
                                         (int)p.n, perr(c));
    });
}

template <typename V>
smash_status run_fused_bins(smash_ctx c, hipStream_t s, const Plan &p)
{
    TRY((launch_fused_bin<V, 6>(c, s, p)));
    TRY((launch_fused_bin<V, 7>(c, s, p)));
    TRY((launch_fused_bin<V, 8>(c, s, p)));
    TRY((launch_fused_bin<V, 9>(c, s, p)));
    TRY((launch_fused_bin<V, 10>(c, s, p)));
    TRY((launch_fused_bin<V, 11>(c, s, p)));
    return SMASH_OK;
}

// Copies the device header (and the numeric error word) to the host and
// waits: the one synchronisation of a symbolic call.
smash_status read_hdr(smash_ctx c, hipStream_t s)
{
    HIP_TRY(c, hipMemcpyAsync(c->h_hdr, c->d_hdr, kNumErrOffset + sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    collect_times(c);
    return SMASH_OK;
}

smash_status device_errors(smash_ctx c, int e)
{
    if (e & (kErrCsrA | kErrCsrB))
        return fail(c, SMASH_ERR_INVALID_CSR, "%s violates the CSR preconditions (row_ptr[0] = 0, nondecreasing, "
                    "row_ptr[rows] = nnz, columns in range and strictly ascending)",
                    (e & kErrCsrA) ? "A" : "B");
    if (e & (kErrProbe | kErrCount))
        return fail(c, SMASH_ERR_CAPACITY, "C_row_ptr does not match the product (device flags 0x%x)", e);
    return SMASH_OK;
}

// Errors recorded by earlier numeric calls (read at a synchronisation):
// reported once, then cleared.
smash_status numeric_errors(smash_ctx c, hipStream_t s)
{
    const int e = *c->h_numerr;
    if (!e) return SMASH_OK;
    *c->h_numerr = 0;
    HIP_TRY(c, hipMemsetAsync(c->d_numerr, 0, sizeof(int), s));
    const smash_status st = device_errors(c, e);
    c->err = std::string(smash_status_string(st)) + ": a numeric call before this one failed on the device: " +
             c->err.substr(c->err.find(": ") + 2);
    return st;
}

// The fused stage of smash_spgemm_fused: predicted capacities, fused bins,
// staging offsets (a synchronisation reads their total, and the staging
// area comes from the caller's allocation callback), the fused kernels, and
// removal of the rows they completed from the two-phase plan.
smash_status fused_stage(smash_ctx c, hipStream_t s, Plan &p, smash_alloc_fn alloc, void *user)
{
    const int m = (int)p.m;
    const size_t vb = p.fused_dtype == SMASH_F32 ? 4 : 8;
    const float *prm = (const float *)c->pred_mem.ptr;
    const bool learned = c->opt[SMASH_OPT_FUSED_SIZING] == 0;
    if (learned) {      // the features came with the analysis
        TRY(launch(c, K_MLP_PREDICT, s, [&] {
            k_mlp_predict<<<blocks_for(m, 256), 256, 0, s>>>(m, (int)p.n, p.feats, prm, prm + kParams,
                                                             c->pred_delta, p.ub, p.maxb, nullptr, p.cap_pred,
                                                             p.lds_row_max);
        }));
    }
    TRY(launch(c, K_FUSED_AUX, s, [&] {
        k_fused_bins<<<blocks_for(m, 256), 256, 0, s>>>(m, p.ub, learned ? p.cap_pred : p.cap, p.lds_row_max,
                                                        p.fbin, p.fcap, perr(c));
    }));
    TRY(bin_rows(c, s, p, p.fbin, nullptr, nullptr, &c->d_hdr->fz, p.f_perm, nullptr, -1));
    TRY(scan_counts<int>(c, s, m, p.fcap, p.bsum, p.stage_off, &c->d_hdr->stage_total));
    TRY(read_hdr(c, s));
    TRY(device_errors(c, c->h_hdr->error));
    const long long total = c->h_hdr->stage_total;
    p.stage_cap = total;
    p.stage_col = (int *)alloc(std::max<size_t>((size_t)total * 4, 256), user);
    p.stage_val = alloc(std::max<size_t>((size_t)total * vb, 256), user);
    if (!p.stage_col || !p.stage_val) return fail(c, SMASH_ERR_OUT_OF_MEMORY, "allocation callback returned NULL");
    if (p.fused_dtype == SMASH_F32) TRY(run_fused_bins<float>(c, s, p));
    else TRY(run_fused_bins<double>(c, s, p));
    TRY(launch(c, K_FUSED_AUX, s, [&] {
        k_fused_mark<<<std::min(blocks_for(m, 256), 1024u), 256, 0, s>>>(m, p.fbin, p.fstatus, p.nnzc, p.sym_bin, &c->d_hdr->fused_ok,
                                                        &c->d_hdr->fused_entries, perr(c));
    }));
    return SMASH_OK;
}

template <typename V>
smash_status fused_copy(smash_ctx c, hipStream_t s, const Plan &p, const int64_t *crp, int32_t *ccol, V *cval)
{
    const int nf = p.hdr.fz.offset[kLdsBins];
    if (!p.fused || nf == 0) return SMASH_OK;
    return launch(c, K_FUSED_COPY, s, [&] {
        k_fused_copy<V><<<blocks_for(nf, 4), 256, 0, s>>>(p.f_perm, nf, p.fstatus, p.stage_off, p.stage_col,
                                                         (const V *)p.stage_val, (const long long *)crp, ccol, cval);
    });
}

}  // namespace

// =================================================================== C ABI

extern "C" {

const char *smash_status_string(smash_status s)
{
    switch (s) {
    case SMASH_OK: return "SMASH_OK";
    case SMASH_ERR_INVALID_ARG: return "SMASH_ERR_INVALID_ARG";
    case SMASH_ERR_INVALID_CSR: return "SMASH_ERR_INVALID_CSR";
    case SMASH_ERR_INDEX_OVERFLOW: return "SMASH_ERR_INDEX_OVERFLOW";
    case SMASH_ERR_CAPACITY: return "SMASH_ERR_CAPACITY";
    case SMASH_ERR_OUT_OF_MEMORY: return "SMASH_ERR_OUT_OF_MEMORY";
    case SMASH_ERR_HIP: return "SMASH_ERR_HIP";
    case SMASH_ERR_NO_PLAN: return "SMASH_ERR_NO_PLAN";
    }
    return "SMASH_ERR_UNKNOWN";
}

smash_status smash_create(smash_ctx *out, int device)
{
    if (!out) return SMASH_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SMASH_ERR_INVALID_ARG;
    smash_ctx c = new (std::nothrow) smash_ctx_s();
    if (!c) return SMASH_ERR_OUT_OF_MEMORY;
    c->device = device;
    DeviceGuard g(device);
    if (!g.ok || hipHostMalloc((void **)&c->h_hdr, kHdrBytes, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return SMASH_ERR_HIP;
    }
    c->h_numerr = (int *)((char *)c->h_hdr + kNumErrOffset);
    if (hipMalloc((void **)&c->d_hdr, kHdrBytes) != hipSuccess ||
        hipMemset(c->d_hdr, 0, kHdrBytes) != hipSuccess) {
        if (c->d_hdr) (void)hipFree(c->d_hdr);
        (void)hipHostFree(c->h_hdr);
        delete c;
        return SMASH_ERR_OUT_OF_MEMORY;
    }
    c->d_numerr = (int *)((char *)c->d_hdr + kNumErrOffset);
    memset(c->h_hdr, 0, sizeof(DevHdr));
    *c->h_numerr = 0;
    if (device < kMaxDevices) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void *ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
                (void)hipGetLastError();
                (void)hipFree(c->d_hdr);
                (void)hipHostFree(c->h_hdr);
                delete c;
                return SMASH_ERR_HIP;
            }
            g_scratch_ptr[device] = ptr;
        }
        c->scratch = g_scratch_ptr[device];
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cus = cus;
    *out = c;
    return SMASH_OK;
}

void smash_destroy(smash_ctx c)
{
    if (!c) return;
    DeviceGuard g(c->device);
    for (Arena *a : {&c->mlp_mem, &c->pred_mem})
        if (a->ptr) (void)hipFree(a->ptr);
    if (c->d_hdr) (void)hipFree(c->d_hdr);      // holds d_numerr too
    if (c->h_hdr) (void)hipHostFree(c->h_hdr);  // holds h_numerr too
    for (auto &p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    delete c;
}

const char *smash_last_error(smash_ctx c) { return c ? c->err.c_str() : "null context"; }

smash_status smash_set_option(smash_ctx c, smash_option opt, int64_t v)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    switch (opt) {
    case SMASH_OPT_VALIDATE:
    case SMASH_OPT_TIMING:
    case SMASH_OPT_FUSED_SIZING:
        if (v != 0 && v != 1) return fail(c, SMASH_ERR_INVALID_ARG, "option %d takes 0 or 1", (int)opt);
        break;
    case SMASH_OPT_LDS_ROW_MAX:
        if (v < 32 || v > 1024) return fail(c, SMASH_ERR_INVALID_ARG, "LDS row max must be in [32, 1024]");
        break;
    case SMASH_OPT_HEAVY_MODE:
        if (v != 0 && v != 1) return fail(c, SMASH_ERR_INVALID_ARG, "heavy mode is 0 (windowed) or 1 (global hash)");
        break;
    case SMASH_OPT_GLOBAL_POOL:
        if (v < 0) return fail(c, SMASH_ERR_INVALID_ARG, "global pool limit must be >= 0 (0 = no limit)");
        break;
    case SMASH_OPT_ROW_HASH:
        if (v != 0 && v != 1) return fail(c, SMASH_ERR_INVALID_ARG, "row hash is 0 (multiplicative) or 1 (order-preserving)");
        break;
    default: return fail(c, SMASH_ERR_INVALID_ARG, "unknown option %d", (int)opt);
    }
    c->opt[opt] = v;
    c->plan.valid = false;
    return SMASH_OK;
}

smash_status smash_get_option(smash_ctx c, smash_option opt, int64_t *v)
{
    if (!c || !v || (int)opt < 0 || (int)opt >= SMASH_OPT_COUNT) return SMASH_ERR_INVALID_ARG;
    *v = c->opt[opt];
    return SMASH_OK;
}

}  // extern "C"

namespace {

// Heavy rows [0, H) of the global mode in waves of consecutive rows whose
// tables fit `limit` slots (goff: device, the H + 1 table offsets, an
// exclusive prefix).  One wave when all tables fit; otherwise the offsets
// are read back and split greedily, a row whose table alone exceeds the
// limit forming a wave of its own.  bounds receives the first row and table
// offset of every wave followed by (H, goff[H]); pool the slots of the
// largest wave.
smash_status plan_global_waves(smash_ctx c, hipStream_t s, const long long *goff, int H, long long total,
                               long long limit, std::vector<std::pair<int, long long>> &bounds, long long &pool)
{
    bounds.clear();
    if (total <= limit) {
        bounds.push_back({0, 0});
        bounds.push_back({H, total});
        pool = total;
        return SMASH_OK;
    }
    std::vector<long long> off((size_t)H + 1);
    HIP_TRY(c, hipMemcpyAsync(off.data(), goff, off.size() * sizeof(long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    pool = 0;
    for (int h = 0; h < H;) {
        int e = h + 1;
        while (e < H && off[e + 1] - off[h] <= limit) ++e;
        bounds.push_back({h, off[h]});
        pool = std::max(pool, off[e] - off[h]);
        h = e;
    }
    bounds.push_back({H, off[H]});
    return SMASH_OK;
}

// Queues the CSR checks of one matrix (k_validate_rows, k_validate_cols)
// on s; a violation sets `flag` in *err.  With `starts` (a bitmap of
// nnz / 32 + 1 words of the workspace) every precondition is checked;
// without it, only what memory safety needs (row pointers, column ranges).
smash_status validate_csr(smash_ctx c, hipStream_t s, const smash_csr &M, int flag, int *err, unsigned *starts)
{
    if (M.rows == 0 && M.nnz == 0) return SMASH_OK;
    const long long words = (M.nnz + 31) / 32 + 1;
    TRY(launch(c, K_VALIDATE, s, [&] {
        if (starts) k_fill_i32<<<blocks_for(words, 256), 256, 0, s>>>(words, (int *)starts, 0);
        k_validate_rows<<<blocks_for(std::max<int64_t>(M.rows, 1), 256), 256, 0, s>>>((int)M.rows, M.nnz, M.row_ptr,
                                                                                      starts, flag, err);
        if (M.nnz > 0)
            k_validate_cols<<<blocks_for(M.nnz, 256), 256, 0, s>>>((int)M.cols, M.nnz, M.col_idx, starts, flag, err);
    }));
    return SMASH_OK;
}

smash_status check_pair(smash_ctx c, const smash_csr *A, const smash_csr *B, bool need_val)
{
    TRY(check_csr(c, A, "A", need_val));
    TRY(check_csr(c, B, "B", need_val));
    if (A->cols != B->rows)
        return fail(c, SMASH_ERR_INVALID_ARG, "A.cols (%lld) != B.rows (%lld)", (long long)A->cols, (long long)B->rows);
    return SMASH_OK;
}

void plan_init(smash_ctx c, Plan &p, const smash_csr *A, const smash_csr *B, bool fuse, int fused_dtype)
{
    p = Plan();
    p.A = *A;
    p.B = *B;
    p.m = A->rows;
    p.n = B->cols;
    p.heavy_mode = (int)c->opt[SMASH_OPT_HEAVY_MODE];
    p.lds_row_max = (int)c->opt[SMASH_OPT_LDS_ROW_MAX];
    p.row_hash = (int)c->opt[SMASH_OPT_ROW_HASH];
    p.nchunks = (int)std::max<int64_t>(1, (p.n + kChunkCols - 1) / kChunkCols);
    p.fused = fuse;
    p.fused_dtype = fuse ? fused_dtype : 0;
}

// Workspace bytes of C = A * B for the context's options: the fixed part
// from the sizes, the heavy-row part from a device pass that counts the
// heavy rows and the global table slots (checked inputs only: row pointers
// and column ranges first).  Synchronises the stream.
smash_status workspace_query(smash_ctx c, const smash_csr *A, const smash_csr *B, bool fuse, size_t *bytes,
                             hipStream_t s)
{
    Plan q;
    plan_init(c, q, A, B, fuse, 0);
    carve_workspace(c, q, nullptr, 0);
    if (q.m == 0) {
        *bytes = q.ws_fixed;
        return SMASH_OK;
    }
    HIP_TRY(c, hipMemsetAsync(c->d_hdr, 0, sizeof(DevHdr), s));
    TRY(validate_csr(c, s, *A, kErrCsrA, perr(c), nullptr));
    TRY(validate_csr(c, s, *B, kErrCsrB, perr(c), nullptr));
    TRY(launch(c, K_WS_QUERY, s, [&] {
        const unsigned grid =
            (unsigned)std::min<long long>(blocks_for(std::max<long long>(q.m, 1), 256 / kRowLanes), 4096);
        k_ws_query<<<grid, 256, 0, s>>>((int)q.m, (int)q.n, q.lds_row_max, A->row_ptr, A->col_idx, B->row_ptr,
                                        c->d_hdr);
    }));
    TRY(read_hdr(c, s));
    TRY(device_errors(c, c->h_hdr->error));
    const long long H = c->h_hdr->q_heavy;
    long long slots = (long long)c->h_hdr->q_gsum;
    const long long lim = c->opt[SMASH_OPT_GLOBAL_POOL];
    if (lim > 0) slots = std::min<long long>(slots, std::max<long long>(lim, (long long)c->h_hdr->q_gmax));
    *bytes = workspace_need(q, H, slots);
    return SMASH_OK;
}

// The symbolic pipeline; with fused_dtype >= 0 it first runs the fused stage
// for the rows the predictor sizes into LDS (smash_spgemm_fused).
smash_status symbolic_impl(smash_ctx c, const smash_csr *A, const smash_csr *B, int64_t *C_row_ptr, int64_t *C_nnz,
                           void *ws, size_t ws_bytes, hipStream_t s, int fused_dtype, smash_alloc_fn alloc, void *user)
{
    const bool fuse = fused_dtype >= 0;
    c->err.clear();
    c->plan.valid = false;
    TRY(check_pair(c, A, B, fuse));
    if (!C_row_ptr || !C_nnz) return fail(c, SMASH_ERR_INVALID_ARG, "C_row_ptr and C_nnz must not be NULL");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, SMASH_ERR_HIP, "hipSetDevice(%d) failed", c->device);

    Plan &p = c->plan;
    plan_init(c, p, A, B, fuse, fused_dtype);
    p.crp = C_row_ptr;
    const int64_t m = p.m;
    c->stats = smash_stats();
    c->stats.rows = m;
    carve_workspace(c, p, nullptr, 0);
    if (ws_bytes < p.ws_fixed || (!ws && p.ws_fixed > 0)) {
        size_t need = p.ws_fixed;
        if (ws_bytes < p.ws_fixed) TRY(workspace_query(c, A, B, fuse, &need, s));
        c->stats.workspace_bytes = (int64_t)need;
        return fail(c, SMASH_ERR_CAPACITY, "the workspace holds %zu bytes; this product needs %zu", ws_bytes, need);
    }
    carve_workspace(c, p, (char *)ws, ws_bytes);
    p.ws = ws;
    p.ws_bytes = ws_bytes;
    c->stats.workspace_bytes = (int64_t)p.ws_fixed;

    HIP_TRY(c, hipMemsetAsync(c->d_hdr, 0, sizeof(DevHdr), s));
    if (c->opt[SMASH_OPT_VALIDATE]) {
        TRY(validate_csr(c, s, *A, kErrCsrA, perr(c), p.valid_bm));
        if (!same_csr(*A, *B)) TRY(validate_csr(c, s, *B, kErrCsrB, perr(c), p.valid_bm));   // A * A: once
    }
    if (m == 0) {
        HIP_TRY(c, hipMemsetAsync(C_row_ptr, 0, sizeof(int64_t), s));
        TRY(read_hdr(c, s));
        TRY(device_errors(c, c->h_hdr->error));
        TRY(numeric_errors(c, s));
        *C_nnz = 0;
        p.hdr = DevHdr();
        p.valid = true;
        return SMASH_OK;
    }

    // a1/a2: products per row (and the predictor's features for the fused
    // pass), bins, rows grouped by bin
    const bool global = p.heavy_mode == 1;
    const bool learned = fuse && c->opt[SMASH_OPT_FUSED_SIZING] == 0;
    TRY(launch(c, K_ANALYZE, s, [&] {
        k_analyze<<<blocks_for(m, 256 / kRowLanes), 256, 0, s>>>(
            (int)m, (int)p.n, p.lds_row_max, A->row_ptr, A->col_idx, B->row_ptr, p.ub, p.cap, p.nnzc, p.sym_bin,
            learned ? p.feats : nullptr, learned ? p.maxb : nullptr, perr(c));
    }));
    if (fuse) TRY(fused_stage(c, s, p, alloc, user));
    TRY(bin_rows(c, s, p, p.sym_bin, p.ub, nullptr, &c->d_hdr->sym, p.sym_perm, global ? p.cap : nullptr,
                 global ? -1 : p.hcap));
    const int *heavy_rows_dev = p.sym_perm;     // + the heavy bin's offset, read on the device

    // a3: symbolic per bin
    TRY(run_sym_bins(c, s, p));
    if (!global && p.hcap > 0) {
        const long long kdim = p.B.rows;
        TRY(launch(c, K_BSPLIT, s, [&] {
            k_bsplit<<<blocks_for(kdim * (p.nchunks + 1), 256), 256, 0, s>>>((int)kdim, p.nchunks, B->row_ptr,
                                                                            B->col_idx, p.bsplit, perr(c));
        }));
        const int nwin = (p.nchunks + kSymWinChunks - 1) / kSymWinChunks;
        TRY(launch(c, K_SYM_HEAVY, s, [&] {
            k_sym_heavy<<<(unsigned)(p.hcap * nwin), kSymHeavyThreads, 0, s>>>(
                A->row_ptr, A->col_idx, B->col_idx, p.bsplit, (long long)(p.nchunks + 1), heavy_rows_dev,
                &c->d_hdr->sym, (int)p.hcap, p.nchunks, p.wcnt, p.nnzc, perr(c));
        }));
    } else if (global) {
        // the waves are planned on the host: the heavy rows' table offsets
        // are read back (a second synchronisation, in global mode only)
        TRY(read_hdr(c, s));
        TRY(device_errors(c, c->h_hdr->error));
        const int H = c->h_hdr->sym.count[kBinHeavy];
        if (H > 0) {
            const int *heavy_rows = p.sym_perm + c->h_hdr->sym.offset[kBinHeavy];
            TRY(scan_counts<long long>(c, s, H, p.gsz, p.bsum, p.goff_sym, (long long *)&c->d_hdr->gneed[0]));
            TRY(read_hdr(c, s));
            const long long total = (long long)c->h_hdr->gneed[0];
            const long long lim = c->opt[SMASH_OPT_GLOBAL_POOL] > 0
                                      ? std::min<long long>(c->opt[SMASH_OPT_GLOBAL_POOL], p.pool_cap)
                                      : p.pool_cap;
            TRY(plan_global_waves(c, s, p.goff_sym, H, total, lim, p.sym_waves, p.sym_pool));
            if (p.sym_pool > p.pool_cap) {
                c->stats.workspace_bytes = (int64_t)workspace_need(p, 0, p.sym_pool);
                return fail(c, SMASH_ERR_CAPACITY, "a heavy row's global table needs %lld slots; the workspace "
                            "holds %lld (%lld bytes needed)", p.sym_pool, p.pool_cap,
                            (long long)c->stats.workspace_bytes);
            }
            for (size_t w = 0; w + 1 < p.sym_waves.size(); ++w) {
                const int h0 = p.sym_waves[w].first, nh = p.sym_waves[w + 1].first - h0;
                const long long base = p.sym_waves[w].second, slots = p.sym_waves[w + 1].second - base;
                TRY(launch(c, K_FILL, s, [&] { k_fill_i32<<<2048, 256, 0, s>>>(slots, p.gkeys, kEmpty); }));
                TRY(launch(c, K_SYM_GLOBAL, s, [&] {
                    k_sym_global<<<nh, kGlobalThreads, 0, s>>>(A->row_ptr, A->col_idx, B->row_ptr, B->col_idx,
                                                               heavy_rows + h0, p.cap, p.goff_sym + h0, base,
                                                               p.gkeys, p.nnzc, perr(c));
                }));
            }
        }
    }

    // a4: C_row_ptr = exclusive scan of the row counts
    TRY(scan_counts<int>(c, s, m, p.nnzc, p.bsum, (long long *)C_row_ptr, &c->d_hdr->nnz_c));
    // numeric plan: bins of the light rows, segments of the heavy rows
    TRY(launch(c, K_NUM_BINS, s, [&] {
        k_num_bins<<<blocks_for(m, 256), 256, 0, s>>>((int)m, p.nnzc, p.sym_bin, p.num_bin);
    }));
    TRY(bin_rows(c, s, p, p.num_bin, nullptr, p.nnzc, &c->d_hdr->num, p.num_perm, global ? p.nnzc : nullptr, -1));
    if (global && c->h_hdr->sym.count[kBinHeavy] > 0)
        TRY(scan_counts<long long>(c, s, c->h_hdr->sym.count[kBinHeavy], p.gsz, p.bsum, p.goff_num,
                                   (long long *)&c->d_hdr->gneed[1]));
    if (!global && p.hcap > 0) {
        const unsigned nhb = blocks_for(p.hcap, 256);
        TRY(launch(c, K_CHUNK_PREFIX, s, [&] {
            k_chunk_prefix<<<blocks_for(p.hcap, 4), 256, 0, s>>>(&c->d_hdr->sym, p.nchunks, p.wcnt, p.woff, perr(c));
        }));
        TRY(launch(c, K_FILL, s, [&] {
            k_fill_i32<<<blocks_for(kSegBins * p.nchunks, 256), 256, 0, s>>>((long long)kSegBins * p.nchunks,
                                                                           p.seg_bcount, 0);
        }));
        TRY(launch(c, K_SEG_PLAN, s, [&] {
            k_seg_plan<<<nhb, 256, 0, s>>>(0, &c->d_hdr->sym, p.sym_perm, p.nchunks, p.wcnt, p.woff, A->row_ptr,
                                           (const long long *)C_row_ptr, p.seg_bcount, &c->d_hdr->seg, p.segs, perr(c));
        }));
        TRY(launch(c, K_SEG_SCAN, s, [&] {
            k_seg_scan<<<1, kWave, 0, s>>>(p.nchunks, p.seg_bcount, &c->d_hdr->seg, perr(c));
        }));
        TRY(launch(c, K_SEG_PLAN, s, [&] {
            k_seg_plan<<<nhb, 256, 0, s>>>(1, &c->d_hdr->sym, p.sym_perm, p.nchunks, p.wcnt, p.woff, A->row_ptr,
                                           (const long long *)C_row_ptr, p.seg_bcount, &c->d_hdr->seg, p.segs, perr(c));
        }));
    }
    TRY(read_hdr(c, s));
    p.hdr = *c->h_hdr;
    const int H = p.hdr.sym.count[kBinHeavy];
    if (p.hdr.error & kErrCapacity) {
        c->stats.workspace_bytes = (int64_t)workspace_need(p, H, 0);
        return fail(c, SMASH_ERR_CAPACITY, "the workspace holds %lld heavy rows, the product has %d "
                    "(%lld bytes needed)", p.hcap, H, (long long)c->stats.workspace_bytes);
    }
    TRY(device_errors(c, p.hdr.error));
    TRY(numeric_errors(c, s));
    if (H > 0 && global) {
        const long long lim = c->opt[SMASH_OPT_GLOBAL_POOL] > 0
                                  ? std::min<long long>(c->opt[SMASH_OPT_GLOBAL_POOL], p.pool_cap)
                                  : p.pool_cap;
        TRY(plan_global_waves(c, s, p.goff_num, H, (long long)p.hdr.gneed[1], lim, p.num_waves, p.num_pool));
        if (p.num_pool > p.pool_cap)     // cannot happen: numeric tables are no larger than symbolic ones
            return fail(c, SMASH_ERR_CAPACITY, "global tables exceed the workspace");
    }
    c->stats.workspace_bytes = (int64_t)(global ? workspace_need(p, 0, std::max(p.sym_pool, p.num_pool))
                                                : workspace_need(p, H, 0));
    *C_nnz = p.hdr.nnz_c;
    c->stats.products = (int64_t)p.hdr.products;
    c->stats.nnz_c = p.hdr.nnz_c;
    c->stats.rows_empty = p.hdr.sym.count[kBinEmpty];
    c->stats.rows_heavy = H;
    c->stats.rows_lds = m - H - p.hdr.sym.count[kBinEmpty];
    c->stats.heavy_segments = global ? 0 : (p.hdr.seg.offset[kSegBins] - p.hdr.seg.count[kSegDense]);
    c->stats.heavy_dense_chunks = global ? 0 : p.hdr.seg.count[kSegDense];
    c->stats.nnz_heavy = p.hdr.num.wsum[kBinHeavy];
    c->stats.nnz_dense = global ? 0 : p.hdr.seg.nnz[kSegDense];
    c->stats.global_slots = global ? (int64_t)(p.hdr.gneed[0] + p.hdr.gneed[1]) : 0;
    c->stats.global_waves = (int64_t)(p.sym_waves.empty() ? 0 : p.sym_waves.size() - 1) +
                            (int64_t)(p.num_waves.empty() ? 0 : p.num_waves.size() - 1);
    c->stats.global_pool = std::max(p.sym_pool, p.num_pool);
    if (fuse) {
        c->stats.fused_rows = p.hdr.fused_ok;
        c->stats.fused_overflow = p.hdr.fz.offset[kLdsBins] - p.hdr.fused_ok;
        c->stats.fused_capacity = p.hdr.stage_total;
        c->stats.fused_entries = (int64_t)p.hdr.fused_entries;
        c->stats.rows_empty -= p.hdr.fused_ok;
    }
    p.valid = true;
    return SMASH_OK;
}

template <typename V>
smash_status numeric_dispatch(smash_ctx c, hipStream_t s, const Plan &p, const smash_csr *A, const smash_csr *B,
                              const int64_t *C_row_ptr, int32_t *C_col_idx, void *C_val)
{
    TRY(numeric_impl<V>(c, s, p, (const V *)A->val, (const V *)B->val, C_row_ptr, C_col_idx, (V *)C_val));
    return fused_copy<V>(c, s, p, C_row_ptr, C_col_idx, (V *)C_val);
}

smash_status numeric_checked(smash_ctx c, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                             const int64_t *C_row_ptr, int32_t *C_col_idx, void *C_val, const void *ws,
                             hipStream_t s)
{
    c->err.clear();
    if (dtype != SMASH_F32 && dtype != SMASH_F64) return fail(c, SMASH_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    TRY(check_csr(c, A, "A", true));
    TRY(check_csr(c, B, "B", true));
    const Plan &p = c->plan;
    if (!p.valid || !same_csr(p.A, *A) || !same_csr(p.B, *B) || p.crp != C_row_ptr || p.ws != ws)
        return fail(c, SMASH_ERR_NO_PLAN, "no symbolic plan on this context for these A, B, C_row_ptr and workspace");
    if (p.fused && (int)dtype != p.fused_dtype) return fail(c, SMASH_ERR_INVALID_ARG, "dtype differs from the fused pass");
    if (p.hdr.nnz_c > 0 && (!C_col_idx || !C_val))
        return fail(c, SMASH_ERR_INVALID_ARG, "C_col_idx and C_val must not be NULL");
    if (p.m == 0 || p.hdr.nnz_c == 0) return SMASH_OK;
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, SMASH_ERR_HIP, "hipSetDevice(%d) failed", c->device);
    if (dtype == SMASH_F32) return numeric_dispatch<float>(c, s, p, A, B, C_row_ptr, C_col_idx, C_val);
    return numeric_dispatch<double>(c, s, p, A, B, C_row_ptr, C_col_idx, C_val);
}

}  // namespace

extern "C" {

smash_status smash_workspace_size(smash_ctx c, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                                  size_t *bytes, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    c->err.clear();
    if (!bytes) return fail(c, SMASH_ERR_INVALID_ARG, "bytes is NULL");
    if (dtype != SMASH_F32 && dtype != SMASH_F64) return fail(c, SMASH_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    TRY(check_pair(c, A, B, false));
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, SMASH_ERR_HIP, "hipSetDevice(%d) failed", c->device);
    size_t plain = 0, fused = 0;
    TRY(workspace_query(c, A, B, false, &plain, s));
    const bool fusable = c->has_predictor || c->opt[SMASH_OPT_FUSED_SIZING] == 1;
    if (fusable) {
        Plan q;
        plan_init(c, q, A, B, true, (int)dtype);
        carve_workspace(c, q, nullptr, 0);
        Plan r;
        plan_init(c, r, A, B, false, 0);
        carve_workspace(c, r, nullptr, 0);
        fused = plain + (q.ws_fixed - r.ws_fixed);
    }
    *bytes = std::max(plain, fused);
    return SMASH_OK;
}

smash_status smash_spgemm_symbolic(smash_ctx c, const smash_csr *A, const smash_csr *B, int64_t *C_row_ptr,
                                   int64_t *C_nnz, void *ws, size_t ws_bytes, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    return symbolic_impl(c, A, B, C_row_ptr, C_nnz, ws, ws_bytes, s, -1, nullptr, nullptr);
}

smash_status smash_spgemm_numeric(smash_ctx c, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                                  const int64_t *C_row_ptr, int32_t *C_col_idx, void *C_val, void *ws,
                                  size_t ws_bytes, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    if (c->plan.fused) return fail(c, SMASH_ERR_NO_PLAN, "the plan belongs to a fused call");
    (void)ws_bytes;
    return numeric_checked(c, dtype, A, B, C_row_ptr, C_col_idx, C_val, ws, s);
}

smash_status smash_spgemm(smash_ctx c, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                          smash_alloc_fn alloc, void *user, int64_t *C_row_ptr, int32_t **C_col_idx, void **C_val,
                          int64_t *C_nnz, void *ws, size_t ws_bytes, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    if (!alloc || !C_col_idx || !C_val || !C_nnz) return fail(c, SMASH_ERR_INVALID_ARG, "null output argument");
    if (dtype != SMASH_F32 && dtype != SMASH_F64) return fail(c, SMASH_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    int64_t nnz = 0;
    TRY(smash_spgemm_symbolic(c, A, B, C_row_ptr, &nnz, ws, ws_bytes, s));
    const size_t vb = dtype == SMASH_F32 ? 4 : 8;
    void *col = alloc(std::max<size_t>((size_t)nnz * 4, 256), user);
    void *val = alloc(std::max<size_t>((size_t)nnz * vb, 256), user);
    if (!col || !val) return fail(c, SMASH_ERR_OUT_OF_MEMORY, "allocation callback returned NULL");
    *C_col_idx = (int32_t *)col;
    *C_val = val;
    *C_nnz = nnz;
    return smash_spgemm_numeric(c, dtype, A, B, C_row_ptr, (int32_t *)col, val, ws, ws_bytes, s);
}

smash_status smash_spgemm_noalloc(smash_ctx c, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                                  int64_t *C_row_ptr, int32_t *C_col_idx, void *C_val, int64_t C_capacity,
                                  int64_t *C_nnz, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    c->err.clear();
    if (!C_nnz || C_capacity < 0) return fail(c, SMASH_ERR_INVALID_ARG, "C_nnz is NULL or C_capacity < 0");
    if (dtype != SMASH_F32 && dtype != SMASH_F64) return fail(c, SMASH_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if (c->opt[SMASH_OPT_HEAVY_MODE] != 0)
        return fail(c, SMASH_ERR_INVALID_ARG, "the no-allocation entry point runs the LDS heavy-row mode only");
    if (!c->scratch) return fail(c, SMASH_ERR_HIP, "no scratch array on device %d", c->device);
    int64_t nnz = 0;
    const smash_status st = symbolic_impl(c, A, B, C_row_ptr, &nnz, c->scratch, kScratchBytes, s, -1, nullptr,
                                          nullptr);
    if (st == SMASH_ERR_CAPACITY)
        return fail(c, SMASH_ERR_CAPACITY, "the product needs %lld bytes of workspace; the no-allocation entry "
                    "point has %zu", (long long)c->stats.workspace_bytes, kScratchBytes);
    if (st != SMASH_OK) return st;
    *C_nnz = nnz;
    if (nnz > C_capacity) {
        c->plan.valid = false;
        return fail(c, SMASH_ERR_CAPACITY, "C has %lld entries; the output buffers hold %lld", (long long)nnz,
                    (long long)C_capacity);
    }
    return numeric_checked(c, dtype, A, B, C_row_ptr, C_col_idx, C_val, c->scratch, s);
}

smash_status smash_sync(smash_ctx c, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    c->err.clear();
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, SMASH_ERR_HIP, "hipSetDevice(%d) failed", c->device);
    HIP_TRY(c, hipMemcpyAsync(c->h_numerr, c->d_numerr, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    collect_times(c);
    const int e = *c->h_numerr;
    if (!e) return SMASH_OK;
    *c->h_numerr = 0;
    HIP_TRY(c, hipMemsetAsync(c->d_numerr, 0, sizeof(int), s));
    return device_errors(c, e);
}

smash_status smash_features(smash_ctx c, const smash_csr *A, const smash_csr *B, float *feats, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    c->err.clear();
    TRY(check_csr(c, A, "A", false));
    TRY(check_csr(c, B, "B", false));
    if (A->cols != B->rows) return fail(c, SMASH_ERR_INVALID_ARG, "A.cols != B.rows");
    if (!feats && A->rows > 0) return fail(c, SMASH_ERR_INVALID_ARG, "feats is NULL");
    if (A->rows == 0) return SMASH_OK;
    DeviceGuard g(c->device);
    TRY(launch(c, K_FEATURES, s, [&] {
        k_features<<<blocks_for(A->rows, 4), 256, 0, s>>>((int)A->rows, (int)B->cols, A->row_ptr, A->col_idx,
                                                          B->row_ptr, feats, nullptr, nullptr);
    }));
    return SMASH_OK;
}

smash_status smash_mlp_predict(smash_ctx c, int64_t m, const float *feats, const float *params, const float *ms,
                               float *yhat, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    c->err.clear();
    if (m < 0 || m >= INT32_MAX) return fail(c, SMASH_ERR_INVALID_ARG, "bad row count");
    if (m == 0) return SMASH_OK;
    if (!feats || !params || !ms || !yhat) return fail(c, SMASH_ERR_INVALID_ARG, "null pointer");
    DeviceGuard g(c->device);
    TRY(launch(c, K_MLP_PREDICT, s, [&] {
        k_mlp_predict<<<blocks_for(m, 256), 256, 0, s>>>((int)m, 0, feats, params, ms, 0.f, nullptr, nullptr, yhat,
                                                         nullptr, -1);
    }));
    return SMASH_OK;
}

}  // extern "C"

namespace {

struct MlpBufs {
    float *h1, *h2, *dz2, *dz1, *dy, *grad, *mom, *vel;
    double *sse;
};

smash_status mlp_bufs(smash_ctx c, hipStream_t s, int batch, long long sse_slots, MlpBufs &b)
{
    const size_t need = carve_size({(size_t)batch * kHid * 4, (size_t)batch * kHid * 4, (size_t)batch * kHid * 4,
                                    (size_t)batch * kHid * 4, (size_t)batch * 4, (size_t)kParams * 4,
                                    (size_t)kParams * 4, (size_t)kParams * 4, (size_t)sse_slots * 8});
    TRY(ensure(c, c->mlp_mem, need, s));
    Carve cv{(char *)c->mlp_mem.ptr};
    b.h1 = cv.take<float>((size_t)batch * kHid);
    b.h2 = cv.take<float>((size_t)batch * kHid);
    b.dz2 = cv.take<float>((size_t)batch * kHid);
    b.dz1 = cv.take<float>((size_t)batch * kHid);
    b.dy = cv.take<float>(batch);
    b.grad = cv.take<float>(kParams);
    b.mom = cv.take<float>(kParams);
    b.vel = cv.take<float>(kParams);
    b.sse = cv.take<double>(sse_slots);
    return SMASH_OK;
}

// Forward and backward of one batch; leaves the gradient in b.grad and the
// block sums of squared errors in sse[0 .. ceil(n/256)).
smash_status mlp_step(smash_ctx c, hipStream_t s, const float *feats, const float *targets, const int *idx, int n,
                      const float *ms, const float *params, MlpBufs &b, double *sse)
{
    TRY(launch(c, K_MLP_FWD, s, [&] {
        k_mlp_fwd<<<blocks_for(n, 256), 256, 0, s>>>(n, idx, feats, targets, ms, params, b.h1, b.h2, b.dy, sse);
    }));
    TRY(launch(c, K_MLP_BWD, s, [&] {
        k_mlp_grad_out<<<kHid + 1, 256, 0, s>>>(n, b.h2, b.dy, params, b.dz2, b.grad);
    }));
    TRY(launch(c, K_MLP_BWD, s, [&] { k_mlp_grad_mid<<<kHid, 256, 0, s>>>(n, b.h1, b.dz2, b.grad); }));
    TRY(launch(c, K_MLP_BWD, s, [&] {
        k_mlp_back_h1<<<blocks_for((long long)n * kHid, 256), 256, 0, s>>>(n, b.h1, b.dz2, params, b.dz1);
    }));
    TRY(launch(c, K_MLP_BWD, s, [&] { k_mlp_grad_in<<<kHid, 256, 0, s>>>(n, idx, feats, ms, b.dz1, b.grad); }));
    return SMASH_OK;
}

}  // namespace

extern "C" {

smash_status smash_mlp_loss_grad(smash_ctx c, const float *feats, const float *targets, const int32_t *idx, int64_t n,
                                 const float *ms, const float *params, float *grad, double *loss, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    c->err.clear();
    if (n <= 0 || n > (1 << 24)) return fail(c, SMASH_ERR_INVALID_ARG, "batch size must be in [1, 2^24]");
    if (!feats || !targets || !idx || !ms || !params || !grad || !loss)
        return fail(c, SMASH_ERR_INVALID_ARG, "null pointer");
    DeviceGuard g(c->device);
    MlpBufs b;
    const int nb = (int)blocks_for(n, 256);
    TRY(mlp_bufs(c, s, (int)n, nb, b));
    TRY(mlp_step(c, s, feats, targets, idx, (int)n, ms, params, b, b.sse));
    HIP_TRY(c, hipMemcpyAsync(grad, b.grad, kParams * sizeof(float), hipMemcpyDeviceToDevice, s));
    std::vector<double> part(nb);
    HIP_TRY(c, hipMemcpyAsync(part.data(), b.sse, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    collect_times(c);
    double tot = 0;
    for (double v : part) tot += v;
    *loss = tot / (double)n;
    return SMASH_OK;
}

smash_status smash_mlp_train(smash_ctx c, const float *feats, const float *targets, int64_t n, const float *ms,
                             float *params, const int32_t *orders, const smash_train_args *a, double *epoch_loss,
                             hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    c->err.clear();
    if (!a || a->epochs <= 0 || a->batch <= 0 || a->batch > (1 << 20) || n <= 0 || n >= INT32_MAX)
        return fail(c, SMASH_ERR_INVALID_ARG, "bad training arguments");
    if (!feats || !targets || !ms || !params || !orders || !epoch_loss)
        return fail(c, SMASH_ERR_INVALID_ARG, "null pointer");
    DeviceGuard g(c->device);
    const int batch = (int)std::min<int64_t>(a->batch, n);
    const int steps = (int)((n + batch - 1) / batch);
    const int nbmax = (int)blocks_for(batch, 256);
    const long long slots = (long long)a->epochs * steps * nbmax;
    MlpBufs b;
    TRY(mlp_bufs(c, s, batch, slots, b));
    HIP_TRY(c, hipMemsetAsync(b.mom, 0, kParams * sizeof(float), s));
    HIP_TRY(c, hipMemsetAsync(b.vel, 0, kParams * sizeof(float), s));
    HIP_TRY(c, hipMemsetAsync(b.sse, 0, slots * sizeof(double), s));
    int t = 0;
    for (int e = 0; e < a->epochs; ++e) {
        for (int st = 0; st < steps; ++st) {
            const int s0 = st * batch;
            const int nb = (int)std::min<int64_t>(batch, n - s0);
            const int *idx = orders + (long long)e * n + s0;
            TRY(mlp_step(c, s, feats, targets, idx, nb, ms, params, b, b.sse + ((long long)e * steps + st) * nbmax));
            ++t;
            TRY(launch(c, K_ADAM, s, [&] {
                k_adam<<<blocks_for(kParams, 256), 256, 0, s>>>(kParams, params, b.grad, b.mom, b.vel, t, a->lr,
                                                               a->beta1, a->beta2, a->eps);
            }));
        }
    }
    std::vector<double> part(slots);
    HIP_TRY(c, hipMemcpyAsync(part.data(), b.sse, slots * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    collect_times(c);
    for (int e = 0; e < a->epochs; ++e) {
        double acc = 0.0;
        for (int st = 0; st < steps; ++st) {
            const int nb = (int)std::min<int64_t>(batch, n - (long long)st * batch);
            double sse = 0.0;
            for (int q = 0; q < nbmax; ++q) sse += part[((long long)e * steps + st) * nbmax + q];
            acc += sse / nb;
        }
        epoch_loss[e] = acc / steps;
    }
    return SMASH_OK;
}

smash_status smash_predictor_set(smash_ctx c, const float *params, const float *ms, float delta)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    c->err.clear();
    if (!params || !ms) return fail(c, SMASH_ERR_INVALID_ARG, "null pointer");
    for (int f = 0; f < kFeat; ++f)
        if (!(ms[kFeat + f] > 0.f)) return fail(c, SMASH_ERR_INVALID_ARG, "feature std must be positive");
    DeviceGuard g(c->device);
    TRY(ensure(c, c->pred_mem, (kParams + 2 * kFeat) * sizeof(float), nullptr));
    HIP_TRY(c, hipMemcpy(c->pred_mem.ptr, params, kParams * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy((float *)c->pred_mem.ptr + kParams, ms, 2 * kFeat * sizeof(float), hipMemcpyHostToDevice));
    c->pred_delta = delta;
    c->has_predictor = true;
    return SMASH_OK;
}

smash_status smash_predictor_load(smash_ctx c, const char *path)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    c->err.clear();
    if (!path) return fail(c, SMASH_ERR_INVALID_ARG, "null path");
    FILE *f = fopen(path, "rb");
    if (!f) return fail(c, SMASH_ERR_INVALID_ARG, "cannot open %s", path);
    char magic[8];
    int32_t ver = 0, np = 0;
    float delta = 0.f;
    std::vector<float> ms(2 * kFeat), prm(kParams);
    const bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "SMASHMLP", 8) == 0 && fread(&ver, 4, 1, f) == 1 &&
                    ver == 1 && fread(&np, 4, 1, f) == 1 && np == kParams && fread(&delta, 4, 1, f) == 1 &&
                    fread(ms.data(), 4, ms.size(), f) == ms.size() && fread(prm.data(), 4, prm.size(), f) == prm.size();
    fclose(f);
    if (!ok) return fail(c, SMASH_ERR_INVALID_ARG, "%s is not a version-1 predictor file", path);
    return smash_predictor_set(c, prm.data(), ms.data(), delta);
}

smash_status smash_spgemm_fused(smash_ctx c, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                                smash_alloc_fn alloc, void *user, int64_t *C_row_ptr, int32_t **C_col_idx,
                                void **C_val, int64_t *C_nnz, void *ws, size_t ws_bytes, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    if (!alloc || !C_col_idx || !C_val || !C_nnz || !C_row_ptr)
        return fail(c, SMASH_ERR_INVALID_ARG, "null output argument");
    if (dtype != SMASH_F32 && dtype != SMASH_F64) return fail(c, SMASH_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if (!c->has_predictor && c->opt[SMASH_OPT_FUSED_SIZING] == 0)
        return fail(c, SMASH_ERR_NO_PLAN, "no predictor installed (smash_predictor_set/load)");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, SMASH_ERR_HIP, "hipSetDevice(%d) failed", c->device);
    int64_t nnz = 0;
    TRY(symbolic_impl(c, A, B, C_row_ptr, &nnz, ws, ws_bytes, s, (int)dtype, alloc, user));
    Plan &p = c->plan;
    const size_t vb = dtype == SMASH_F32 ? 4 : 8;
    void *col = alloc(std::max<size_t>((size_t)nnz * 4, 256), user);
    void *val = alloc(std::max<size_t>((size_t)nnz * vb, 256), user);
    if (!col || !val) {
        p.valid = false;
        return fail(c, SMASH_ERR_OUT_OF_MEMORY, "allocation callback returned NULL");
    }
    *C_col_idx = (int32_t *)col;
    *C_val = val;
    *C_nnz = nnz;
    const smash_status st = numeric_checked(c, dtype, A, B, C_row_ptr, (int32_t *)col, val, ws, s);
    p.valid = false;    // the staged values belong to this call only
    return st;
}

smash_status smash_get_stats(smash_ctx c, smash_stats *out)
{
    if (!c || !out) return SMASH_ERR_INVALID_ARG;
    *out = c->stats;
    return SMASH_OK;
}

int smash_kernel_count(void) { return K_COUNT; }

smash_status smash_kernel_time(smash_ctx c, int index, const char **name, int64_t *launches, double *ms)
{
    if (!c || index < 0 || index >= K_COUNT) return SMASH_ERR_INVALID_ARG;
    collect_times(c);
    if (name) *name = kKernelNames[index];
    if (launches) *launches = c->launches[index];
    if (ms) *ms = c->ms[index];
    return SMASH_OK;
}

smash_status smash_kernel_time_reset(smash_ctx c)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    collect_times(c);
    for (int k = 0; k < K_COUNT; ++k) {
        c->launches[k] = 0;
        c->ms[k] = 0.0;
    }
    return SMASH_OK;
}

}  // extern "C"


// ======================================================= batched launch

struct smash_batch_plan_s {
    smash_ctx c = nullptr;
    smash_dtype dtype = SMASH_F32;
    int count = 0;
    long long M = 0;                     // rows of all problems
    long long nnz_a = 0, nnz_b = 0;
    unsigned long long products = 0;
    smash_batch_config cfg{};
    int ncu = 256;
    std::vector<BatchDesc> desc;
    std::vector<int64_t> row0;           // count + 1
    // workspace (caller-owned, from the allocation callback)
    smash_alloc_fn alloc = nullptr;
    void *user = nullptr;
    void *ws = nullptr;
    unsigned *valid_bm = nullptr;
    BatchDesc *d_desc = nullptr;
    long long *d_row0 = nullptr, *ub = nullptr, *gsz = nullptr, *goff = nullptr, *bsum = nullptr, *pnnz = nullptr;
    int *prob = nullptr, *cap = nullptr, *nnzc = nullptr, *sym_perm = nullptr, *num_perm = nullptr, *bcount = nullptr;
    unsigned char *sym_bin = nullptr, *num_bin = nullptr;
    unsigned long long *bprod = nullptr;
    RowDesc *rd = nullptr;               // row records of the LDS bins
    int nblk = 0;
    BatchHdr *d_hdr = nullptr, *h_hdr = nullptr;
    int *gkeys = nullptr, *gtouch = nullptr;
    double *gvals = nullptr;
    long long gcap = 0;                  // slots of gkeys / gvals / gtouch
    long long cap_total = 0;             // sum of the row bounds (pool capacity)
    int wide_words = 1;                  // LDS bitmap words of the widest problem up to kWideMaxCols
    bool any_global = false;             // a problem wider than kWideMaxCols (global tables)
    // caller-owned output pool
    long long *crp = nullptr;
    int *ccol = nullptr;
    void *cval = nullptr;
    long long ccap = 0;
    hipGraphExec_t exec = nullptr;
};

namespace {

using BPlan = smash_batch_plan_s;

bool batch_cfg_ok(const smash_batch_config &g)
{
    return g.lds_row_max >= 32 && g.lds_row_max <= 1024 && (g.table_shift == 1 || g.table_shift == 2) &&
           g.lds_row_max <= (2048 >> g.table_shift) && (g.wide_groups == 0 || g.wide_groups == 1) &&
           g.blocks_per_cu >= 1 && g.blocks_per_cu <= 32 && (g.row_hash == 0 || g.row_hash == 1);
}

template <int LOGT, int WIDE>
struct BShape {
    static constexpr int WPR = WIDE ? (LOGT <= 8 ? 1 : 1 << (LOGT - 8)) : (LOGT <= 10 ? 1 : 1 << (LOGT - 9));
    static constexpr int RPW = WPR == 1 ? 4 : 1;
    static constexpr int THREADS = kWave * WPR * RPW;
};

unsigned bgrid(const BPlan &p, long long items)
{
    const long long g = (long long)p.cfg.blocks_per_cu * p.ncu;
    return (unsigned)std::max<long long>(1, std::min<long long>(g, items));
}

template <typename TIn>
void bscan(const BPlan &p, hipStream_t s, long long n, const TIn *in, long long *out, long long *total)
{
    const int nb = (int)blocks_for(std::max<long long>(n, 1), kScanItems);
    k_scan_reduce<TIn><<<nb, kScanThreads, 0, s>>>(n, in, p.bsum);
    k_scan_top<<<1, kScanThreads, 0, s>>>(nb, p.bsum, total);
    k_scan_apply<TIn><<<nb, kScanThreads, 0, s>>>(n, in, p.bsum, total, out);
}

void bbin(const BPlan &p, hipStream_t s, const unsigned char *bin_of, BinHdr *h, int *perm, bool products)
{
    const int m = (int)p.M;
    k_bin_count<<<p.nblk, 256, 0, s>>>(m, bin_of, products ? p.ub : nullptr, nullptr, p.bcount,
                                       products ? p.bprod : nullptr, nullptr, nullptr);
    k_bin_scan<<<1, 256, 0, s>>>(p.nblk, p.bcount, products ? p.bprod : nullptr, nullptr, h,
                                 products ? &p.d_hdr->products : nullptr, nullptr, -1);
    k_scatter<<<p.nblk, 256, 0, s>>>(m, bin_of, p.bcount, h, perm, nullptr, nullptr, nullptr);
}

// clears the header and runs the per-row analysis (graph-safe)
void batch_analyze(const BPlan &p, hipStream_t s)
{
    k_fill_i32<<<1, 256, 0, s>>>((long long)(sizeof(BatchHdr) / sizeof(int)), (int *)p.d_hdr, 0);
    k_banalyze<<<bgrid(p, blocks_for(p.M, 4 * kWave)), 256, 0, s>>>(p.M, p.count, p.d_row0, p.d_desc, p.cfg.lds_row_max,
                                                            p.cfg.table_shift, p.prob, p.ub, p.cap, p.nnzc,
                                                            p.sym_bin, p.gsz);
}

template <int LT, int WIDE>
void bsym_bin(const BPlan &p, hipStream_t s)
{
    using S = BShape<LT, WIDE>;
    k_bsym_rows<LT, S::WPR, S::RPW><<<bgrid(p, blocks_for(p.M, S::RPW)), S::THREADS, 0, s>>>(
        p.d_desc, p.rd, &p.d_hdr->sym, LT - kMinLogT, p.nnzc, &p.d_hdr->error);
}

template <typename V, int LT, int WIDE>
void bnum_bin(const BPlan &p, hipStream_t s)
{
    using S = BShape<LT, WIDE>;
    const unsigned grid = bgrid(p, blocks_for(p.M, S::RPW));
    if (p.cfg.row_hash)
        k_bnum_rows<V, LT, S::WPR, S::RPW, 1><<<grid, S::THREADS, 0, s>>>(p.d_desc, p.rd, p.d_hdr, LT - kMinLogT,
                                                                         p.ccap, p.ccol, (V *)p.cval, &p.d_hdr->error);
    else
        k_bnum_rows<V, LT, S::WPR, S::RPW, 0><<<grid, S::THREADS, 0, s>>>(p.d_desc, p.rd, p.d_hdr, LT - kMinLogT,
                                                                         p.ccap, p.ccol, (V *)p.cval, &p.d_hdr->error);
}

template <int WIDE>
void bsym_bins(const BPlan &p, hipStream_t s)
{
    bsym_bin<6, WIDE>(p, s);
    bsym_bin<7, WIDE>(p, s);
    bsym_bin<8, WIDE>(p, s);
    bsym_bin<9, WIDE>(p, s);
    bsym_bin<10, WIDE>(p, s);
    bsym_bin<11, WIDE>(p, s);
}

template <typename V, int WIDE>
void bnum_bins(const BPlan &p, hipStream_t s)
{
    bnum_bin<V, 6, WIDE>(p, s);
    bnum_bin<V, 7, WIDE>(p, s);
    bnum_bin<V, 8, WIDE>(p, s);
    bnum_bin<V, 9, WIDE>(p, s);
    bnum_bin<V, 10, WIDE>(p, s);
    bnum_bin<V, 11, WIDE>(p, s);
}

template <typename V>
void batch_numeric(const BPlan &p, hipStream_t s)
{
    if (p.cfg.wide_groups) bnum_bins<V, 1>(p, s);
    else bnum_bins<V, 0>(p, s);
    k_bnum_wide<V><<<bgrid(p, p.M), kWideThreads, kWideWin * sizeof(double), s>>>(
        p.d_desc, p.prob, p.d_hdr, p.num_perm, p.ccap, p.crp, p.ccol, (V *)p.cval, &p.d_hdr->error,
        &p.d_hdr->wide_queue);
    if (p.any_global)
        k_bnum_global<V><<<bgrid(p, p.M), kGlobalThreads, kGlobalRankBits / 8, s>>>(
        p.d_desc, p.prob, p.d_hdr, p.num_perm, p.goff, p.gcap, p.gkeys, p.gvals, p.gtouch, p.ccap, p.crp, p.ccol,
        (V *)p.cval, &p.d_hdr->error);
}

// the whole batch: no host synchronisation, no allocation, no memset
void batch_enqueue(const BPlan &p, hipStream_t s)
{
    if (p.M == 0) {     // nothing to compute; keeps a captured graph non-empty
        k_fill_i32<<<1, 256, 0, s>>>((long long)(sizeof(BatchHdr) / sizeof(int)), (int *)p.d_hdr, 0);
        return;
    }
    batch_analyze(p, s);
    bbin(p, s, p.sym_bin, &p.d_hdr->sym, p.sym_perm, true);
    bscan<long long>(p, s, p.M, p.gsz, p.goff, &p.d_hdr->gneed);
    k_browdesc<<<bgrid(p, blocks_for(p.M, 256)), 256, 0, s>>>(p.d_desc, p.prob, &p.d_hdr->sym, p.sym_perm, nullptr,
                                                               p.rd);
    if (p.cfg.wide_groups) bsym_bins<1>(p, s);
    else bsym_bins<0>(p, s);
    k_bsym_wide<<<bgrid(p, p.M), kWideThreads, p.wide_words * sizeof(unsigned), s>>>(
        p.d_desc, p.prob, &p.d_hdr->sym, p.sym_perm, p.nnzc);
    if (p.any_global)
        k_bsym_global<<<bgrid(p, p.M), kGlobalThreads, 0, s>>>(p.d_desc, p.prob, &p.d_hdr->sym, p.sym_perm, p.cap,
                                                           p.goff, p.gcap, p.gkeys, p.nnzc, &p.d_hdr->error);
    bscan<int>(p, s, p.M, p.nnzc, p.crp, &p.d_hdr->nnz_c);
    k_bcheck<<<1, 64, 0, s>>>(p.d_hdr, p.ccap);
    k_bnum_bins<<<bgrid(p, blocks_for(p.M, 256)), 256, 0, s>>>(p.M, p.cfg.table_shift, p.nnzc, p.sym_bin,
                                                               p.num_bin);
    bbin(p, s, p.num_bin, &p.d_hdr->num, p.num_perm, false);
    k_browdesc<<<bgrid(p, blocks_for(p.M, 256)), 256, 0, s>>>(p.d_desc, p.prob, &p.d_hdr->num, p.num_perm, p.crp,
                                                               p.rd);
    if (p.dtype == SMASH_F32) batch_numeric<float>(p, s);
    else batch_numeric<double>(p, s);
}

smash_status batch_sync(BPlan &p, hipStream_t s)
{
    HIP_TRY(p.c, hipGetLastError());
    HIP_TRY(p.c, hipMemcpyAsync(p.h_hdr, p.d_hdr, sizeof(BatchHdr), hipMemcpyDeviceToHost, s));
    HIP_TRY(p.c, hipStreamSynchronize(s));
    return SMASH_OK;
}

// sizes the global tables for the plan's configuration (analysis + scan)
smash_status batch_size_tables(BPlan &p, hipStream_t s)
{
    if (p.M == 0) return SMASH_OK;
    batch_analyze(p, s);
    bscan<long long>(p, s, p.M, p.gsz, p.goff, &p.d_hdr->gneed);
    TRY(batch_sync(p, s));
    const long long need = std::max<long long>(p.h_hdr->gneed, 1);
    if (need > p.gcap) {
        // larger tables from the caller's allocation callback (the caller
        // keeps owning the smaller ones it handed out before)
        p.gkeys = (int *)p.alloc((size_t)need * sizeof(int), p.user);
        p.gvals = (double *)p.alloc((size_t)need * sizeof(double), p.user);
        p.gtouch = (int *)p.alloc((size_t)need * sizeof(int), p.user);
        p.gcap = 0;
        if (!p.gkeys || !p.gvals || !p.gtouch)
            return fail(p.c, SMASH_ERR_OUT_OF_MEMORY, "global tables of %lld slots", need);
        p.gcap = need;
    }
    if (p.exec) {
        (void)hipGraphExecDestroy(p.exec);
        p.exec = nullptr;
    }
    return SMASH_OK;
}

void batch_free(BPlan *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->h_hdr) (void)hipHostFree(p->h_hdr);
    delete p;
}

}  // namespace

extern "C" {

smash_status smash_batch_plan_create(smash_ctx c, smash_dtype dtype, int32_t count, const smash_csr *A,
                                     const smash_csr *B, const smash_batch_config *cfg, smash_alloc_fn alloc,
                                     void *user, smash_batch_plan *out, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    c->err.clear();
    if (!out || !alloc || count < 0 || (count > 0 && (!A || !B)))
        return fail(c, SMASH_ERR_INVALID_ARG, "NULL argument or negative count");
    *out = nullptr;
    if (dtype != SMASH_F32 && dtype != SMASH_F64) return fail(c, SMASH_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    const smash_batch_config def{1024, 1, 0, 8, 0};
    const smash_batch_config g = cfg ? *cfg : def;
    if (!batch_cfg_ok(g)) return fail(c, SMASH_ERR_INVALID_ARG, "batch configuration out of range");
    for (int q = 0; q < count; ++q) {
        TRY(check_csr(c, &A[q], "A", true));
        TRY(check_csr(c, &B[q], "B", true));
        if (A[q].cols != B[q].rows)
            return fail(c, SMASH_ERR_INVALID_ARG, "problem %d: A.cols (%lld) != B.rows (%lld)", q,
                        (long long)A[q].cols, (long long)B[q].rows);
    }
    DeviceGuard dg(c->device);
    if (!dg.ok) return fail(c, SMASH_ERR_HIP, "hipSetDevice(%d) failed", c->device);
    BPlan *p = new (std::nothrow) BPlan();
    if (!p) return fail(c, SMASH_ERR_OUT_OF_MEMORY, "plan");
    p->c = c;
    p->dtype = dtype;
    p->count = count;
    p->cfg = g;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && ncu > 0)
        p->ncu = ncu;
    p->row0.assign((size_t)count + 1, 0);
    p->desc.resize((size_t)std::max(count, 1));
    for (int q = 0; q < count; ++q) {
        p->row0[q + 1] = p->row0[q] + A[q].rows;
        p->nnz_a += A[q].nnz;
        p->nnz_b += B[q].nnz;
        p->desc[q] = BatchDesc{A[q].row_ptr, A[q].col_idx, A[q].val, B[q].row_ptr, B[q].col_idx, B[q].val,
                               (int)A[q].rows, (int)B[q].cols, (long long)p->row0[q]};
    }
    p->M = p->row0[count];
    for (int q = 0; q < count; ++q) {
        if (B[q].cols <= kWideMaxCols) p->wide_words = std::max(p->wide_words, (int)((B[q].cols + 31) / 32));
        else p->any_global = true;
    }
    smash_status st = SMASH_OK;
    auto bail = [&](smash_status e) {
        batch_free(p);
        return e;
    };
    if (p->M >= (1LL << 31) - 1) return bail(fail(c, SMASH_ERR_INDEX_OVERFLOW, "batch of %lld rows", p->M));
    const long long M = std::max<long long>(p->M, 1);
    p->nblk = (int)blocks_for(M, kBinBlockRows);
    const int nsb = (int)blocks_for(M, kScanItems);
    long long max_nnz = 0;
    for (int q = 0; q < count; ++q) max_nnz = std::max<long long>(max_nnz, std::max(A[q].nnz, B[q].nnz));
    const size_t bm_words = (size_t)(max_nnz + 31) / 32 + 1;
    const size_t need = carve_size({p->desc.size() * sizeof(BatchDesc), ((size_t)count + 1) * 8, (size_t)M * 4,
                                    (size_t)M * 8, (size_t)M * 4, (size_t)M * 4, (size_t)M, (size_t)M,
                                    (size_t)M * 8, (size_t)(M + 1) * 8, (size_t)M * 4, (size_t)M * 4,
                                    (size_t)p->nblk * kNumBins * 4, (size_t)p->nblk * 8, (size_t)(nsb + 1) * 8,
                                    (size_t)std::max(count, 1) * 8, sizeof(BatchHdr), (size_t)M * sizeof(RowDesc),
                                    bm_words * 4});
    // the plan's workspace and, later, its global tables come from the
    // caller's allocation callback: the library allocates no device memory
    p->alloc = alloc;
    p->user = user;
    p->ws = alloc(need, user);
    if (!p->ws) return bail(fail(c, SMASH_ERR_OUT_OF_MEMORY, "allocation callback returned NULL (workspace)"));
    if (hipHostMalloc((void **)&p->h_hdr, sizeof(BatchHdr), hipHostMallocDefault) != hipSuccess)
        return bail(fail(c, SMASH_ERR_HIP, "pinned header"));
    if (hipFuncSetAttribute((const void *)k_bsym_wide, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(p->wide_words * sizeof(unsigned))) != hipSuccess ||
        hipFuncSetAttribute((const void *)k_bnum_global<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kGlobalRankBits / 8) != hipSuccess ||
        hipFuncSetAttribute((const void *)k_bnum_global<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kGlobalRankBits / 8) != hipSuccess ||
        hipFuncSetAttribute((const void *)k_bnum_wide<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(kWideWin * sizeof(double))) != hipSuccess ||
        hipFuncSetAttribute((const void *)k_bnum_wide<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(kWideWin * sizeof(double))) != hipSuccess)
        return bail(fail(c, SMASH_ERR_HIP, "hipFuncSetAttribute"));
    Carve cv{(char *)p->ws};
    p->d_desc = cv.take<BatchDesc>(p->desc.size());
    p->d_row0 = cv.take<long long>((size_t)count + 1);
    p->prob = cv.take<int>(M);
    p->ub = cv.take<long long>(M);
    p->cap = cv.take<int>(M);
    p->nnzc = cv.take<int>(M);
    p->sym_bin = cv.take<unsigned char>(M);
    p->num_bin = cv.take<unsigned char>(M);
    p->gsz = cv.take<long long>(M);
    p->goff = cv.take<long long>(M + 1);
    p->sym_perm = cv.take<int>(M);
    p->num_perm = cv.take<int>(M);
    p->bcount = cv.take<int>((size_t)p->nblk * kNumBins);
    p->bprod = cv.take<unsigned long long>(p->nblk);
    p->bsum = cv.take<long long>(nsb + 1);
    p->pnnz = cv.take<long long>(std::max(count, 1));
    p->d_hdr = cv.take<BatchHdr>(1);
    p->rd = cv.take<RowDesc>(M);
    p->valid_bm = cv.take<unsigned>(bm_words);
    if (hipMemcpyAsync(p->d_desc, p->desc.data(), p->desc.size() * sizeof(BatchDesc), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(p->d_row0, p->row0.data(), ((size_t)count + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess)
        return bail(fail(c, SMASH_ERR_HIP, "descriptor upload"));
    if (c->opt[SMASH_OPT_VALIDATE] && count > 0) {
        k_fill_i32<<<1, 256, 0, s>>>((long long)(sizeof(BatchHdr) / sizeof(int)), (int *)p->d_hdr, 0);
        for (int q = 0; q < count && st == SMASH_OK; ++q) {
            st = validate_csr(c, s, A[q], kErrCsrA, &p->d_hdr->error, p->valid_bm);
            if (st == SMASH_OK) st = validate_csr(c, s, B[q], kErrCsrB, &p->d_hdr->error, p->valid_bm);
        }
        if (st != SMASH_OK) return bail(st);
        st = batch_sync(*p, s);
        if (st != SMASH_OK) return bail(st);
        if (p->h_hdr->error)
            return bail(fail(c, SMASH_ERR_INVALID_CSR, "an operand of the batch violates the CSR preconditions"));
    }
    // output pool: sum over rows of min(ub, cols)
    if (p->M > 0) {
        batch_analyze(*p, s);
        bscan<int>(*p, s, p->M, p->cap, p->goff, &p->d_hdr->nnz_c);
        st = batch_sync(*p, s);
        if (st != SMASH_OK) return bail(st);
        p->cap_total = p->h_hdr->nnz_c;
    }
    st = batch_size_tables(*p, s);
    if (st != SMASH_OK) return bail(st);
    const size_t vb = dtype == SMASH_F32 ? 4 : 8;
    p->ccap = p->cap_total;
    p->crp = (long long *)alloc((size_t)(p->M + 1) * 8, user);
    p->ccol = (int *)alloc(std::max<size_t>((size_t)p->ccap * 4, 256), user);
    p->cval = alloc(std::max<size_t>((size_t)p->ccap * vb, 256), user);
    if (!p->crp || !p->ccol || !p->cval) return bail(fail(c, SMASH_ERR_OUT_OF_MEMORY, "allocation callback failed"));
    if (p->M == 0 && hipMemsetAsync(p->crp, 0, 8, s) != hipSuccess) return bail(fail(c, SMASH_ERR_HIP, "memset"));
    // products of the batch
    if (p->M > 0) {
        bbin(*p, s, p->sym_bin, &p->d_hdr->sym, p->sym_perm, true);
        st = batch_sync(*p, s);
        if (st != SMASH_OK) return bail(st);
        p->products = p->h_hdr->products;
    }
    *out = p;
    return SMASH_OK;
}

smash_status smash_batch_plan_configure(smash_batch_plan p, const smash_batch_config *cfg, hipStream_t s)
{
    if (!p || !cfg) return SMASH_ERR_INVALID_ARG;
    if (!batch_cfg_ok(*cfg)) return fail(p->c, SMASH_ERR_INVALID_ARG, "batch configuration out of range");
    DeviceGuard dg(p->c->device);
    if (!dg.ok) return fail(p->c, SMASH_ERR_HIP, "hipSetDevice failed");
    p->cfg = *cfg;
    return batch_size_tables(*p, s);
}

smash_status smash_batch_plan_get_config(smash_batch_plan p, smash_batch_config *cfg)
{
    if (!p || !cfg) return SMASH_ERR_INVALID_ARG;
    *cfg = p->cfg;
    return SMASH_OK;
}

smash_status smash_batch_plan_outputs(smash_batch_plan p, int64_t **C_row_ptr, int32_t **C_col_idx, void **C_val,
                                      int64_t *capacity, int64_t *total_rows, const int64_t **row0)
{
    if (!p) return SMASH_ERR_INVALID_ARG;
    if (C_row_ptr) *C_row_ptr = (int64_t *)p->crp;
    if (C_col_idx) *C_col_idx = p->ccol;
    if (C_val) *C_val = p->cval;
    if (capacity) *capacity = p->ccap;
    if (total_rows) *total_rows = p->M;
    if (row0) *row0 = p->row0.data();
    return SMASH_OK;
}

smash_status smash_batch_plan_run(smash_batch_plan p, hipStream_t s)
{
    if (!p) return SMASH_ERR_INVALID_ARG;
    DeviceGuard dg(p->c->device);
    if (!dg.ok) return fail(p->c, SMASH_ERR_HIP, "hipSetDevice failed");
    batch_enqueue(*p, s);
    HIP_TRY(p->c, hipGetLastError());
    return SMASH_OK;
}

smash_status smash_batch_plan_capture(smash_batch_plan p, hipStream_t s)
{
    if (!p) return SMASH_ERR_INVALID_ARG;
    DeviceGuard dg(p->c->device);
    if (!dg.ok) return fail(p->c, SMASH_ERR_HIP, "hipSetDevice failed");
    if (p->exec) {
        (void)hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    HIP_TRY(p->c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    batch_enqueue(*p, s);
    const hipError_t launch_err = hipGetLastError();
    HIP_TRY(p->c, hipStreamEndCapture(s, &graph));
    if (launch_err != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(p->c, SMASH_ERR_HIP, "launch during capture: %s", hipGetErrorString(launch_err));
    }
    const hipError_t e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        p->exec = nullptr;
        return fail(p->c, SMASH_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return SMASH_OK;
}

smash_status smash_batch_plan_launch(smash_batch_plan p, hipStream_t s)
{
    if (!p) return SMASH_ERR_INVALID_ARG;
    if (!p->exec) return fail(p->c, SMASH_ERR_NO_PLAN, "no captured graph on this plan");
    DeviceGuard dg(p->c->device);
    if (!dg.ok) return fail(p->c, SMASH_ERR_HIP, "hipSetDevice failed");
    HIP_TRY(p->c, hipGraphLaunch(p->exec, s));
    return SMASH_OK;
}

smash_status smash_batch_plan_result(smash_batch_plan p, hipStream_t s, int64_t *nnz_total, int64_t *nnz_per_problem)
{
    if (!p) return SMASH_ERR_INVALID_ARG;
    DeviceGuard dg(p->c->device);
    if (!dg.ok) return fail(p->c, SMASH_ERR_HIP, "hipSetDevice failed");
    if (p->M == 0) {
        if (nnz_total) *nnz_total = 0;
        if (nnz_per_problem)
            for (int q = 0; q < p->count; ++q) nnz_per_problem[q] = 0;
        return SMASH_OK;
    }
    if (nnz_per_problem && p->count > 0) {
        k_bproblem_nnz<<<blocks_for(p->count, 256), 256, 0, s>>>(p->count, p->d_row0, p->crp, p->pnnz);
        HIP_TRY(p->c, hipMemcpyAsync(nnz_per_problem, p->pnnz, (size_t)p->count * 8, hipMemcpyDeviceToHost, s));
    }
    TRY(batch_sync(*p, s));
    const int e = p->h_hdr->error;
    if (nnz_total) *nnz_total = p->h_hdr->nnz_c;
    if (e & kErrCapacity)
        return fail(p->c, SMASH_ERR_CAPACITY, "the batch needs %lld entries (or more global table slots) beyond "
                    "the plan's pool of %lld", (long long)p->h_hdr->nnz_c, p->ccap);
    if (e) return fail(p->c, SMASH_ERR_HIP, "internal inconsistency (device error flags 0x%x)", e);
    return SMASH_OK;
}

void smash_batch_plan_destroy(smash_batch_plan p)
{
    if (!p) return;
    DeviceGuard dg(p->c->device);
    batch_free(p);
}

smash_status smash_batch_autotune(smash_batch_plan p, hipStream_t s, int32_t reps, const char *cache_path,
                                  smash_batch_config *best, double *best_ms)
{
    if (!p || reps < 1) return SMASH_ERR_INVALID_ARG;
    DeviceGuard dg(p->c->device);
    if (!dg.ok) return fail(p->c, SMASH_ERR_HIP, "hipSetDevice failed");
    char key[256];
    snprintf(key, sizeof key, "%s:%d:%lld:%lld:%lld:%llu", p->dtype == SMASH_F32 ? "f32" : "f64", p->count, p->M,
             p->nnz_a, p->nnz_b, p->products);
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "r")) {
            char k[256];
            smash_batch_config g{};
            double ms = 0;
            bool hit = false;
            smash_batch_config found{};
            while (fscanf(f, "%255s %d %d %d %d %d %lf", k, &g.lds_row_max, &g.table_shift, &g.wide_groups,
                          &g.blocks_per_cu, &g.row_hash, &ms) == 7)
                if (strcmp(k, key) == 0 && batch_cfg_ok(g)) {
                    found = g;
                    hit = true;
                }
            fclose(f);
            if (hit) {
                TRY(smash_batch_plan_configure(p, &found, s));
                if (best) *best = found;
                if (best_ms) *best_ms = 0.0;
                return SMASH_OK;
            }
        }
    }
    std::vector<smash_batch_config> cands;
    for (int lrm : {256, 512, 1024})
        for (int sh : {1, 2})
            for (int wide : {0, 1})
                for (int bpc : {4, 16})
                    for (int rh : {0, 1}) {
                        const smash_batch_config g{lrm, sh, wide, bpc, rh};
                        if (batch_cfg_ok(g)) cands.push_back(g);
                    }
    hipEvent_t e0, e1;
    HIP_TRY(p->c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(p->c, SMASH_ERR_HIP, "hipEventCreate");
    }
    smash_status st = SMASH_OK;
    double top = 1e300;
    smash_batch_config win = p->cfg;
    for (const smash_batch_config &g : cands) {
        st = smash_batch_plan_configure(p, &g, s);
        if (st != SMASH_OK) break;
        batch_enqueue(*p, s);                      // warm-up
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) batch_enqueue(*p, s);
        (void)hipEventRecord(e1, s);
        st = smash_batch_plan_result(p, s, nullptr, nullptr);
        if (st != SMASH_OK) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double per = ms / reps;
        if (per < top) {
            top = per;
            win = g;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SMASH_OK) return st;
    TRY(smash_batch_plan_configure(p, &win, s));
    if (best) *best = win;
    if (best_ms) *best_ms = top;
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (!f) return fail(p->c, SMASH_ERR_INVALID_ARG, "cannot append to %s", cache_path);
        fprintf(f, "%s %d %d %d %d %d %.6f\n", key, win.lds_row_max, win.table_shift, win.wide_groups,
                win.blocks_per_cu, win.row_hash, top);
        fclose(f);
    }
    return SMASH_OK;
}

}  // extern "C"
