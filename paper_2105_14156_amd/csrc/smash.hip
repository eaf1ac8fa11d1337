// smash.hip -- host side of libsmash: contexts, planning, launches and the C
// ABI declared in include/smash.h.
//
// Call structure (SMASH Kernels chapter: window distribution, hashing and
// write-back phases, each closed by a barrier; here every phase is a set of
// kernels ordered on the caller's stream):
//   symbolic: validate -> analyze (products per row, bins) -> bin offsets ->
//             scatter rows by bin -> [read bin counts back] -> per-bin LDS
//             hash kernels + heavy-row kernel -> row-pointer scan -> numeric
//             bins -> [read nnz(C) back]
//   numeric:  per-bin LDS hash kernels (hash, compact, sort, write) +
//             heavy-row kernels -> [read error flags back]
#include "smash.h"
#include "smash_kernels.hpp"
#include "smash_mlp.hpp"
#include "smash_fused.hpp"
#include "smash_batch.hpp"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

using namespace smash;

namespace {

enum KernelId {
    K_VALIDATE, K_ANALYZE, K_BIN_COUNT, K_BIN_SCAN, K_SCATTER, K_SYM_ROWS, K_BSPLIT, K_SYM_HEAVY,
    K_SYM_GLOBAL, K_FILL, K_SCAN_REDUCE, K_SCAN_TOP, K_SCAN_APPLY, K_NUM_BINS, K_CHUNK_PREFIX,
    K_SEG_PLAN, K_SEG_SCAN, K_NUM_ROWS, K_NUM_SEG, K_NUM_DENSE, K_NUM_GLOBAL, K_FEATURES, K_MLP_PREDICT,
    K_MLP_FWD, K_MLP_BWD, K_ADAM, K_FUSED_ROWS, K_FUSED_AUX, K_FUSED_COPY, K_COUNT
};

const char *const kKernelNames[K_COUNT] = {
    "validate", "analyze", "bin_count", "bin_scan", "scatter", "sym_rows", "bsplit", "sym_heavy",
    "sym_global", "fill", "scan_reduce", "scan_top", "scan_apply", "num_bins", "chunk_prefix",
    "seg_plan", "seg_scan", "num_rows", "num_seg", "num_dense", "num_global", "features", "mlp_predict",
    "mlp_fwd", "mlp_bwd", "adam", "fused_rows", "fused_aux", "fused_copy"};

// Grow-only device buffer.
struct Arena {
    void *ptr = nullptr;
    size_t cap = 0;
};

struct Carve {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T *p = (T *)(base + off);
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

struct Plan {
    bool valid = false;
    smash_csr A{}, B{};
    const int64_t *crp = nullptr;
    int64_t m = 0, n = 0;
    int heavy_mode = 0, lds_row_max = 0;
    DevHdr hdr{};
    int nchunks = 0, nblk = 0;
    long long *ub = nullptr;
    int *cap = nullptr, *nnzc = nullptr, *sym_perm = nullptr, *num_perm = nullptr;
    unsigned char *sym_bin = nullptr, *num_bin = nullptr;
    int *bcount = nullptr;
    unsigned long long *bprod = nullptr;
    long long *bw = nullptr;
    long long *bsum = nullptr, *gsz = nullptr, *goff_sym = nullptr, *goff_num = nullptr;
    int *bsplit = nullptr, *wcnt = nullptr, *woff = nullptr, *seg_bcount = nullptr;
    Seg *segs = nullptr;
    int *queue = nullptr;                 // work-queue counter of the persistent dense kernel
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
    int *stage_col = nullptr;
    void *stage_val = nullptr;
};

struct Pending {
    int kid;
    hipEvent_t a, b;
};

}  // namespace

struct smash_ctx_s {
    int device = 0;
    std::string err;
    int64_t opt[SMASH_OPT_COUNT] = {1, 1024, 0, 0, 0, 0};
    DevHdr *h_hdr = nullptr;   // pinned host mirror
    DevHdr *d_hdr = nullptr;
    Arena plan_mem, heavy_mem, gkeys, gvals, mlp_mem, pred_mem, fused_mem, stage_mem, valid_mem;
    bool has_predictor = false;
    float pred_delta = 0.f;
    Plan plan;
    smash_stats stats{};
    std::vector<hipEvent_t> event_pool;
    std::vector<Pending> pending;
    int64_t launches[K_COUNT] = {};
    double ms[K_COUNT] = {};
    int cus = 256;                 // compute units of the device
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

// Launches `fn` (a lambda issuing one kernel) and, with timing on, brackets
// it with events on the same stream.
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

// Folds completed timing events into the per-kernel totals (after a sync).
void collect_times(smash_ctx c)
{
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

// ------------------------------------------------------------- LDS bins

template <int LOGT>
struct BinShape {
    // up to 512 slots: a wave per row, four rows per block; 1024 slots: two
    // waves; 2048 slots: four waves
    static constexpr int WPR = LOGT <= 9 ? 1 : (1 << (LOGT - 9));
    static constexpr int RPW = WPR == 1 ? 4 : 1;
    static constexpr int THREADS = kWave * WPR * RPW;
};

template <int LOGT>
smash_status launch_sym_bin(smash_ctx c, hipStream_t s, const Plan &p, int cnt, const int *rows)
{
    using S = BinShape<LOGT>;
    return launch(c, K_SYM_ROWS, s, [&] {
        k_sym_rows<LOGT, S::WPR, S::RPW><<<blocks_for(cnt, S::RPW), S::THREADS, 0, s>>>(
            p.A.row_ptr, p.A.col_idx, p.B.row_ptr, p.B.col_idx, rows, cnt, p.nnzc, &c->d_hdr->error);
    });
}

template <typename V, int LOGT>
smash_status launch_num_bin(smash_ctx c, hipStream_t s, const Plan &p, int cnt, const int *rows, const V *Aval,
                            const V *Bval, const int64_t *crp, int32_t *ccol, V *cval)
{
    using S = BinShape<LOGT>;
    return launch(c, K_NUM_ROWS, s, [&] {
        k_num_rows<V, LOGT, S::WPR, S::RPW><<<blocks_for(cnt, S::RPW), S::THREADS, 0, s>>>(
            p.A.row_ptr, p.A.col_idx, Aval, p.B.row_ptr, p.B.col_idx, Bval, rows, cnt, (const long long *)crp, ccol,
            cval, (int)p.n, &c->d_hdr->error);
    });
}

smash_status run_sym_bins(smash_ctx c, hipStream_t s, const Plan &p)
{
    const BinHdr &b = p.hdr.sym;
    const int *perm = p.sym_perm;
#define SYM_BIN(LT)                                                                               \
    if (b.count[LT - kMinLogT]) TRY(launch_sym_bin<LT>(c, s, p, b.count[LT - kMinLogT], perm + b.offset[LT - kMinLogT]));
    SYM_BIN(6) SYM_BIN(7) SYM_BIN(8) SYM_BIN(9) SYM_BIN(10) SYM_BIN(11)
#undef SYM_BIN
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
// gsize_of is given.
smash_status bin_rows(smash_ctx c, hipStream_t s, const Plan &p, const unsigned char *bin_of, const long long *ub,
                      const int *wt, BinHdr *dh, int *perm, const int *gsize_of)
{
    const int m = (int)p.m;
    TRY(launch(c, K_BIN_COUNT, s, [&] {
        k_bin_count<<<p.nblk, 256, 0, s>>>(m, bin_of, ub, wt, p.bcount, ub ? p.bprod : nullptr, wt ? p.bw : nullptr);
    }));
    TRY(launch(c, K_BIN_SCAN, s, [&] {
        k_bin_scan<<<1, 256, 0, s>>>(p.nblk, p.bcount, ub ? p.bprod : nullptr, wt ? p.bw : nullptr, dh,
                                     ub ? &c->d_hdr->products : nullptr);
    }));
    TRY(launch(c, K_SCATTER, s, [&] {
        k_scatter<<<p.nblk, 256, 0, s>>>(m, bin_of, p.bcount, dh, perm, gsize_of, p.gsz);
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
                                                     cval, &c->d_hdr->error);
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
        // segments of up to 128 and 700 entries (tables of 256 and 1024 slots):
        // two waves each; up to 1024 entries (2048 slots): four
        TRY(launch_seg_bin<V, 8, 128>(c, s, p, 0, Aval, Bval, crp, ccol, cval));
        TRY(launch_seg_bin<V, 10, 128>(c, s, p, 1, Aval, Bval, crp, ccol, cval));
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
                                                               &c->d_hdr->error, nd, p.queue);
            }));
        }
        return SMASH_OK;
    }
    // global-memory hash tables, in the waves planned by the symbolic phase
    // (each row clears its own table, so the pool is reused as it is)
    TRY(ensure(c, c->gkeys, (size_t)p.num_pool * sizeof(int), s));
    TRY(ensure(c, c->gvals, (size_t)p.num_pool * sizeof(V), s));
    const size_t lds = (size_t)kGlobalRankBits / 8;
    (void)hipFuncSetAttribute((const void *)k_num_global<V>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int *rows = p.num_perm + p.hdr.num.offset[kBinHeavy];
    for (size_t w = 0; w + 1 < p.num_waves.size(); ++w) {
        const int h0 = p.num_waves[w].first, nh = p.num_waves[w + 1].first - h0;
        const long long base = p.num_waves[w].second;
        TRY(launch(c, K_NUM_GLOBAL, s, [&] {
            k_num_global<V><<<nh, kGlobalThreads, lds, s>>>(p.A.row_ptr, p.A.col_idx, Aval, p.B.row_ptr, p.B.col_idx,
                                                            Bval, rows + h0, (int)p.n, p.goff_num + h0, base,
                                                            (int *)c->gkeys.ptr, (V *)c->gvals.ptr,
                                                            (const long long *)crp, ccol, cval, &c->d_hdr->error);
        }));
    }
    return SMASH_OK;
}

template <typename V, int LOGT>
smash_status launch_fused_bin(smash_ctx c, hipStream_t s, const Plan &p, int cnt, const int *rows)
{
    using S = BinShape<LOGT>;
    return launch(c, K_FUSED_ROWS, s, [&] {
        k_fused_rows<V, LOGT, S::WPR, S::RPW><<<blocks_for(cnt, S::RPW), S::THREADS, 0, s>>>(
            p.A.row_ptr, p.A.col_idx, (const V *)p.A.val, p.B.row_ptr, p.B.col_idx, (const V *)p.B.val, rows, cnt,
            p.fcap, p.stage_off, p.stage_col, (V *)p.stage_val, p.nnzc, p.fstatus, (int)p.n);
    });
}

template <typename V>
smash_status run_fused_bins(smash_ctx c, hipStream_t s, const Plan &p, const BinHdr &b)
{
#define FUSED_BIN(LT)                                                                                  \
    if (b.count[LT - kMinLogT])                                                                        \
        TRY(launch_fused_bin<V, LT>(c, s, p, b.count[LT - kMinLogT], p.f_perm + b.offset[LT - kMinLogT]));
    FUSED_BIN(6) FUSED_BIN(7) FUSED_BIN(8) FUSED_BIN(9) FUSED_BIN(10) FUSED_BIN(11)
#undef FUSED_BIN
    return SMASH_OK;
}

smash_status bin_rows(smash_ctx c, hipStream_t s, const Plan &p, const unsigned char *bin_of, const long long *ub,
                      const int *wt, BinHdr *dh, int *perm, const int *gsize_of);
template <typename TIn>
smash_status scan_counts(smash_ctx c, hipStream_t s, long long n, const TIn *cnt, long long *bsum, long long *out,
                         long long *total);
smash_status read_hdr(smash_ctx c, hipStream_t s);

// The fused stage of smash_spgemm_fused: features, predicted capacities,
// fused bins, staging offsets, the fused kernels, and removal of the rows
// they completed from the two-phase plan.
smash_status fused_alloc(smash_ctx c, hipStream_t s, Plan &p)
{
    const int m = (int)p.m;
    const size_t need = carve_size({(size_t)m * kFeat * 4, (size_t)m * 4, (size_t)m * 4, (size_t)m * 4,
                                    (size_t)m * 4, (size_t)m, (size_t)m, (size_t)(m + 1) * 8});
    TRY(ensure(c, c->fused_mem, need, s));
    Carve cv{(char *)c->fused_mem.ptr};
    p.feats = cv.take<float>((size_t)m * kFeat);
    p.maxb = cv.take<int>(m);
    p.cap_pred = cv.take<int>(m);
    p.fcap = cv.take<int>(m);
    p.f_perm = cv.take<int>(m);
    p.fbin = cv.take<unsigned char>(m);
    p.fstatus = cv.take<unsigned char>(m);
    p.stage_off = cv.take<long long>(m + 1);
    return SMASH_OK;
}

smash_status fused_stage(smash_ctx c, hipStream_t s, Plan &p)
{
    const int m = (int)p.m;
    const size_t vb = p.fused_dtype == SMASH_F32 ? 4 : 8;
    const float *prm = (const float *)c->pred_mem.ptr;
    const bool learned = c->opt[SMASH_OPT_FUSED_SIZING] == 0;
    if (learned) {      // the features came with the analysis
        TRY(launch(c, K_MLP_PREDICT, s, [&] {
            k_mlp_predict<<<blocks_for(m, 256), 256, 0, s>>>(m, (int)p.n, p.feats, prm, prm + kParams,
                                                             c->pred_delta, p.ub, p.maxb, nullptr, p.cap_pred);
        }));
    }
    TRY(launch(c, K_FUSED_AUX, s, [&] {
        k_fused_bins<<<blocks_for(m, 256), 256, 0, s>>>(m, p.ub, learned ? p.cap_pred : p.cap, p.lds_row_max,
                                                        p.fbin, p.fcap);
    }));
    TRY(bin_rows(c, s, p, p.fbin, nullptr, nullptr, &c->d_hdr->fz, p.f_perm, nullptr));
    TRY(scan_counts<int>(c, s, m, p.fcap, p.bsum, p.stage_off, &c->d_hdr->stage_total));
    TRY(read_hdr(c, s));
    const BinHdr fz = c->h_hdr->fz;
    const long long total = c->h_hdr->stage_total;
    TRY(ensure(c, c->stage_mem, carve_size({(size_t)total * 4, (size_t)total * vb}), s));
    Carve sv{(char *)c->stage_mem.ptr};
    p.stage_col = sv.take<int>(total);
    p.stage_val = sv.take<char>(total * vb);
    if (p.fused_dtype == SMASH_F32) TRY(run_fused_bins<float>(c, s, p, fz));
    else TRY(run_fused_bins<double>(c, s, p, fz));
    TRY(launch(c, K_FUSED_AUX, s, [&] {
        k_fused_mark<<<blocks_for(m, 256), 256, 0, s>>>(m, p.fbin, p.fstatus, p.nnzc, p.sym_bin, &c->d_hdr->fused_ok,
                                                        &c->d_hdr->fused_entries);
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

smash_status read_hdr(smash_ctx c, hipStream_t s)
{
    HIP_TRY(c, hipMemcpyAsync(c->h_hdr, c->d_hdr, sizeof(DevHdr), hipMemcpyDeviceToHost, s));
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
    if (!g.ok || hipHostMalloc((void **)&c->h_hdr, sizeof(DevHdr), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return SMASH_ERR_HIP;
    }
    if (hipMalloc((void **)&c->d_hdr, sizeof(DevHdr)) != hipSuccess) {
        (void)hipHostFree(c->h_hdr);
        delete c;
        return SMASH_ERR_OUT_OF_MEMORY;
    }
    memset(c->h_hdr, 0, sizeof(DevHdr));
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
    for (Arena *a : {&c->plan_mem, &c->heavy_mem, &c->gkeys, &c->gvals, &c->mlp_mem, &c->pred_mem, &c->fused_mem,
                     &c->stage_mem, &c->valid_mem})
        if (a->ptr) (void)hipFree(a->ptr);
    if (c->d_hdr) (void)hipFree(c->d_hdr);
    if (c->h_hdr) (void)hipHostFree(c->h_hdr);
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

namespace {

// Heavy rows [0, H) of the global mode in waves of consecutive rows whose
// tables fit `limit` slots (goff: device, the H + 1 table offsets, an
// exclusive prefix).  One wave without a limit or when all tables fit;
// otherwise the offsets are read back and split greedily, a row whose table
// alone exceeds the limit forming a wave of its own.  bounds receives the
// first row and table offset of every wave followed by (H, goff[H]); pool
// the slots of the largest wave.
smash_status plan_global_waves(smash_ctx c, hipStream_t s, const long long *goff, int H, long long total,
                               int64_t limit, std::vector<std::pair<int, long long>> &bounds, long long &pool)
{
    bounds.clear();
    if (limit <= 0 || total <= limit) {
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
// on s; a violation sets `flag` in *err.  The row-start bitmap lives in the
// context's validation arena (the stream orders successive checks).
smash_status validate_csr(smash_ctx c, hipStream_t s, const smash_csr &M, int flag, int *err)
{
    if (M.rows == 0 && M.nnz == 0) return SMASH_OK;
    const long long words = (M.nnz + 31) / 32 + 1;
    TRY(ensure(c, c->valid_mem, (size_t)words * sizeof(unsigned), s));
    unsigned *starts = (unsigned *)c->valid_mem.ptr;
    TRY(launch(c, K_VALIDATE, s, [&] {
        k_fill_i32<<<blocks_for(words, 256), 256, 0, s>>>(words, (int *)starts, 0);
        k_validate_rows<<<blocks_for(std::max<int64_t>(M.rows, 1), 256), 256, 0, s>>>((int)M.rows, M.nnz, M.row_ptr,
                                                                                      starts, flag, err);
        if (M.nnz > 0)
            k_validate_cols<<<blocks_for(M.nnz, 256), 256, 0, s>>>((int)M.cols, M.nnz, M.col_idx, starts, flag, err);
    }));
    return SMASH_OK;
}

// The symbolic pipeline; with fused_dtype >= 0 it first runs the fused stage
// for the rows the predictor sizes into LDS (smash_spgemm_fused).
smash_status symbolic_impl(smash_ctx c, const smash_csr *A, const smash_csr *B, int64_t *C_row_ptr, int64_t *C_nnz,
                           hipStream_t s, int fused_dtype)
{
    const bool fuse = fused_dtype >= 0;
    c->err.clear();
    c->plan.valid = false;
    TRY(check_csr(c, A, "A", fuse));
    TRY(check_csr(c, B, "B", fuse));
    if (A->cols != B->rows) return fail(c, SMASH_ERR_INVALID_ARG, "A.cols (%lld) != B.rows (%lld)", (long long)A->cols, (long long)B->rows);
    if (!C_row_ptr || !C_nnz) return fail(c, SMASH_ERR_INVALID_ARG, "C_row_ptr and C_nnz must not be NULL");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, SMASH_ERR_HIP, "hipSetDevice(%d) failed", c->device);

    Plan &p = c->plan;
    p = Plan();
    p.A = *A;
    p.B = *B;
    p.crp = C_row_ptr;
    p.m = A->rows;
    p.n = B->cols;
    p.heavy_mode = (int)c->opt[SMASH_OPT_HEAVY_MODE];
    p.lds_row_max = (int)c->opt[SMASH_OPT_LDS_ROW_MAX];
    p.nchunks = (int)std::max<int64_t>(1, (p.n + kChunkCols - 1) / kChunkCols);
    p.fused = fuse;
    p.fused_dtype = fuse ? fused_dtype : 0;
    const int64_t m = p.m;
    c->stats = smash_stats();
    c->stats.rows = m;

    HIP_TRY(c, hipMemsetAsync(c->d_hdr, 0, sizeof(DevHdr), s));
    if (c->opt[SMASH_OPT_VALIDATE]) {
        TRY(validate_csr(c, s, *A, kErrCsrA, &c->d_hdr->error));
        TRY(validate_csr(c, s, *B, kErrCsrB, &c->d_hdr->error));
    }
    if (c->opt[SMASH_OPT_VALIDATE] && m > 0) {
        // no kernel below may dereference an index of an invalid matrix
        TRY(read_hdr(c, s));
        TRY(device_errors(c, c->h_hdr->error));
    }
    if (m == 0) {
        HIP_TRY(c, hipMemsetAsync(C_row_ptr, 0, sizeof(int64_t), s));
        TRY(read_hdr(c, s));
        TRY(device_errors(c, c->h_hdr->error));
        *C_nnz = 0;
        p.hdr = DevHdr();
        p.valid = true;
        return SMASH_OK;
    }

    // per-row plan arrays
    const bool global = p.heavy_mode == 1;
    p.nblk = (int)blocks_for(m, kBinBlockRows);
    const int nsb = (int)blocks_for(m, kScanItems);
    {
        const size_t need = carve_size({m * sizeof(long long), m * sizeof(int), m * sizeof(int), m * sizeof(int),
                                        m * sizeof(int), (size_t)m, (size_t)m,
                                        (size_t)p.nblk * kNumBins * sizeof(int), (size_t)p.nblk * 8,
                                        (size_t)p.nblk * kNumBins * 8,
                                        (size_t)(nsb + 1) * 8, global ? (size_t)m * 8 : 0,
                                        global ? (size_t)(m + 1) * 8 : 0, global ? (size_t)(m + 1) * 8 : 0});
        TRY(ensure(c, c->plan_mem, need, s));
        Carve cv{(char *)c->plan_mem.ptr};
        p.ub = cv.take<long long>(m);
        p.cap = cv.take<int>(m);
        p.nnzc = cv.take<int>(m);
        p.sym_perm = cv.take<int>(m);
        p.num_perm = cv.take<int>(m);
        p.sym_bin = cv.take<unsigned char>(m);
        p.num_bin = cv.take<unsigned char>(m);
        p.bcount = cv.take<int>((size_t)p.nblk * kNumBins);
        p.bprod = cv.take<unsigned long long>(p.nblk);
        p.bw = cv.take<long long>((size_t)p.nblk * kNumBins);
        p.bsum = cv.take<long long>(nsb + 1);
        if (global) {
            p.gsz = cv.take<long long>(m);
            p.goff_sym = cv.take<long long>(m + 1);
            p.goff_num = cv.take<long long>(m + 1);
        }
    }

    // a1/a2: products per row (and the predictor's features for the fused
    // pass), bins, rows grouped by bin
    const bool learned = fuse && c->opt[SMASH_OPT_FUSED_SIZING] == 0;
    if (fuse) TRY(fused_alloc(c, s, p));
    TRY(launch(c, K_ANALYZE, s, [&] {
        k_analyze<<<blocks_for(m, 4), 256, 0, s>>>((int)m, (int)p.n, p.lds_row_max, A->row_ptr, A->col_idx, B->row_ptr,
                                                   p.ub, p.cap, p.nnzc, p.sym_bin, learned ? p.feats : nullptr,
                                                   learned ? p.maxb : nullptr);
    }));
    if (fuse) TRY(fused_stage(c, s, p));
    TRY(bin_rows(c, s, p, p.sym_bin, p.ub, nullptr, &c->d_hdr->sym, p.sym_perm, global ? p.cap : nullptr));
    TRY(read_hdr(c, s));
    TRY(device_errors(c, c->h_hdr->error));
    p.hdr = *c->h_hdr;
    const int H = p.hdr.sym.count[kBinHeavy];
    const int *heavy_rows = p.sym_perm + p.hdr.sym.offset[kBinHeavy];
    if (global && H > 0)
        TRY(scan_counts<long long>(c, s, H, p.gsz, p.bsum, p.goff_sym, (long long *)&c->d_hdr->gneed[0]));

    // a3: symbolic per bin
    TRY(run_sym_bins(c, s, p));
    if (H > 0 && !global) {
        const long long kdim = p.B.rows;
        const size_t cells = (size_t)H * p.nchunks;
        const size_t need = carve_size({(size_t)(kdim * (p.nchunks + 1)) * sizeof(int), cells * sizeof(int),
                                        cells * sizeof(int), (size_t)kSegBins * p.nchunks * sizeof(int),
                                        cells * sizeof(Seg), 64 * sizeof(int)});
        TRY(ensure(c, c->heavy_mem, need, s));
        Carve cv{(char *)c->heavy_mem.ptr};
        p.bsplit = cv.take<int>((size_t)(kdim * (p.nchunks + 1)));
        p.wcnt = cv.take<int>(cells);
        p.woff = cv.take<int>(cells);
        p.seg_bcount = cv.take<int>((size_t)kSegBins * p.nchunks);
        p.segs = cv.take<Seg>(cells);
        p.queue = cv.take<int>(64);
        TRY(launch(c, K_BSPLIT, s, [&] {
            k_bsplit<<<blocks_for(kdim * (p.nchunks + 1), 256), 256, 0, s>>>((int)kdim, p.nchunks, B->row_ptr,
                                                                            B->col_idx, p.bsplit);
        }));
        const int nwin = (p.nchunks + kSymWinChunks - 1) / kSymWinChunks;
        TRY(launch(c, K_SYM_HEAVY, s, [&] {
            k_sym_heavy<<<(unsigned)((long long)H * nwin), kSymHeavyThreads, 0, s>>>(
                A->row_ptr, A->col_idx, B->col_idx, p.bsplit, (long long)(p.nchunks + 1), heavy_rows, H, p.nchunks, p.wcnt, p.nnzc);
        }));
    } else if (H > 0) {
        TRY(read_hdr(c, s));
        TRY(plan_global_waves(c, s, p.goff_sym, H, (long long)c->h_hdr->gneed[0], c->opt[SMASH_OPT_GLOBAL_POOL],
                              p.sym_waves, p.sym_pool));
        TRY(ensure(c, c->gkeys, (size_t)p.sym_pool * sizeof(int), s));
        for (size_t w = 0; w + 1 < p.sym_waves.size(); ++w) {
            const int h0 = p.sym_waves[w].first, nh = p.sym_waves[w + 1].first - h0;
            const long long base = p.sym_waves[w].second, slots = p.sym_waves[w + 1].second - base;
            TRY(launch(c, K_FILL, s, [&] { k_fill_i32<<<2048, 256, 0, s>>>(slots, (int *)c->gkeys.ptr, kEmpty); }));
            TRY(launch(c, K_SYM_GLOBAL, s, [&] {
                k_sym_global<<<nh, kGlobalThreads, 0, s>>>(A->row_ptr, A->col_idx, B->row_ptr, B->col_idx,
                                                           heavy_rows + h0, p.cap, p.goff_sym + h0, base,
                                                           (int *)c->gkeys.ptr, p.nnzc, &c->d_hdr->error);
            }));
        }
    }

    // a4: C_row_ptr = exclusive scan of the row counts
    TRY(scan_counts<int>(c, s, m, p.nnzc, p.bsum, (long long *)C_row_ptr, &c->d_hdr->nnz_c));
    // numeric plan: bins of the light rows, segments of the heavy rows
    TRY(launch(c, K_NUM_BINS, s, [&] {
        k_num_bins<<<blocks_for(m, 256), 256, 0, s>>>((int)m, p.nnzc, p.sym_bin, p.num_bin);
    }));
    TRY(bin_rows(c, s, p, p.num_bin, nullptr, p.nnzc, &c->d_hdr->num, p.num_perm, global ? p.nnzc : nullptr));
    if (H > 0 && global)
        TRY(scan_counts<long long>(c, s, H, p.gsz, p.bsum, p.goff_num, (long long *)&c->d_hdr->gneed[1]));
    if (H > 0 && !global) {
        const int nhb = (int)blocks_for(H, 256);
        TRY(launch(c, K_CHUNK_PREFIX, s, [&] {
            k_chunk_prefix<<<blocks_for(H, 4), 256, 0, s>>>(H, p.nchunks, p.wcnt, p.woff);
        }));
        TRY(launch(c, K_FILL, s, [&] {
            k_fill_i32<<<blocks_for(kSegBins * p.nchunks, 256), 256, 0, s>>>((long long)kSegBins * p.nchunks,
                                                                           p.seg_bcount, 0);
        }));
        TRY(launch(c, K_SEG_PLAN, s, [&] {
            k_seg_plan<<<nhb, 256, 0, s>>>(0, H, p.nchunks, p.wcnt, p.woff, heavy_rows, A->row_ptr,
                                           (const long long *)C_row_ptr, p.seg_bcount, &c->d_hdr->seg, p.segs);
        }));
        TRY(launch(c, K_SEG_SCAN, s, [&] { k_seg_scan<<<1, kWave, 0, s>>>(p.nchunks, p.seg_bcount, &c->d_hdr->seg); }));
        TRY(launch(c, K_SEG_PLAN, s, [&] {
            k_seg_plan<<<nhb, 256, 0, s>>>(1, H, p.nchunks, p.wcnt, p.woff, heavy_rows, A->row_ptr,
                                           (const long long *)C_row_ptr, p.seg_bcount, &c->d_hdr->seg, p.segs);
        }));
    }
    TRY(read_hdr(c, s));
    p.hdr = *c->h_hdr;
    TRY(device_errors(c, p.hdr.error));
    if (H > 0 && global)
        TRY(plan_global_waves(c, s, p.goff_num, H, (long long)p.hdr.gneed[1], c->opt[SMASH_OPT_GLOBAL_POOL],
                              p.num_waves, p.num_pool));
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

}  // namespace

smash_status smash_spgemm_symbolic(smash_ctx c, const smash_csr *A, const smash_csr *B, int64_t *C_row_ptr,
                                   int64_t *C_nnz, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    return symbolic_impl(c, A, B, C_row_ptr, C_nnz, s, -1);
}

smash_status smash_spgemm_numeric(smash_ctx c, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                                  const int64_t *C_row_ptr, int32_t *C_col_idx, void *C_val, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    c->err.clear();
    if (dtype != SMASH_F32 && dtype != SMASH_F64) return fail(c, SMASH_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    TRY(check_csr(c, A, "A", true));
    TRY(check_csr(c, B, "B", true));
    const Plan &p = c->plan;
    if (!p.valid || p.fused || !same_csr(p.A, *A) || !same_csr(p.B, *B) || p.crp != C_row_ptr)
        return fail(c, SMASH_ERR_NO_PLAN, "no symbolic plan on this context for these A, B and C_row_ptr");
    if (p.hdr.nnz_c > 0 && (!C_col_idx || !C_val))
        return fail(c, SMASH_ERR_INVALID_ARG, "C_col_idx and C_val must not be NULL");
    if (p.m == 0 || p.hdr.nnz_c == 0) return SMASH_OK;
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, SMASH_ERR_HIP, "hipSetDevice(%d) failed", c->device);
    HIP_TRY(c, hipMemsetAsync(&c->d_hdr->error, 0, sizeof(int), s));
    smash_status st;
    if (dtype == SMASH_F32)
        st = numeric_impl<float>(c, s, p, (const float *)A->val, (const float *)B->val, C_row_ptr, C_col_idx,
                                 (float *)C_val);
    else
        st = numeric_impl<double>(c, s, p, (const double *)A->val, (const double *)B->val, C_row_ptr, C_col_idx,
                                  (double *)C_val);
    if (st != SMASH_OK) return st;
    TRY(read_hdr(c, s));
    return device_errors(c, c->h_hdr->error);
}

smash_status smash_spgemm(smash_ctx c, smash_dtype dtype, const smash_csr *A, const smash_csr *B,
                          smash_alloc_fn alloc, void *user, int64_t *C_row_ptr, int32_t **C_col_idx, void **C_val,
                          int64_t *C_nnz, hipStream_t s)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
    if (!alloc || !C_col_idx || !C_val || !C_nnz) return fail(c, SMASH_ERR_INVALID_ARG, "null output argument");
    if (dtype != SMASH_F32 && dtype != SMASH_F64) return fail(c, SMASH_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    int64_t nnz = 0;
    TRY(smash_spgemm_symbolic(c, A, B, C_row_ptr, &nnz, s));
    const size_t vb = dtype == SMASH_F32 ? 4 : 8;
    void *col = alloc(std::max<size_t>((size_t)nnz * 4, 256), user);
    void *val = alloc(std::max<size_t>((size_t)nnz * vb, 256), user);
    if (!col || !val) return fail(c, SMASH_ERR_OUT_OF_MEMORY, "allocation callback returned NULL");
    *C_col_idx = (int32_t *)col;
    *C_val = val;
    *C_nnz = nnz;
    return smash_spgemm_numeric(c, dtype, A, B, C_row_ptr, (int32_t *)col, val, s);
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
                                                         nullptr);
    }));
    return SMASH_OK;
}

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
                                void **C_val, int64_t *C_nnz, hipStream_t s)
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
    TRY(symbolic_impl(c, A, B, C_row_ptr, &nnz, s, (int)dtype));
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
    smash_status st = SMASH_OK;
    if (p.m > 0 && nnz > 0) {
        HIP_TRY(c, hipMemsetAsync(&c->d_hdr->error, 0, sizeof(int), s));
        if (dtype == SMASH_F32) {
            st = numeric_impl<float>(c, s, p, (const float *)A->val, (const float *)B->val, C_row_ptr, (int32_t *)col,
                                     (float *)val);
            if (st == SMASH_OK) st = fused_copy<float>(c, s, p, C_row_ptr, (int32_t *)col, (float *)val);
        } else {
            st = numeric_impl<double>(c, s, p, (const double *)A->val, (const double *)B->val, C_row_ptr,
                                      (int32_t *)col, (double *)val);
            if (st == SMASH_OK) st = fused_copy<double>(c, s, p, C_row_ptr, (int32_t *)col, (double *)val);
        }
        if (st == SMASH_OK) st = read_hdr(c, s);
        if (st == SMASH_OK) st = device_errors(c, c->h_hdr->error);
    }
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
    if (name) *name = kKernelNames[index];
    if (launches) *launches = c->launches[index];
    if (ms) *ms = c->ms[index];
    return SMASH_OK;
}

smash_status smash_kernel_time_reset(smash_ctx c)
{
    if (!c) return SMASH_ERR_INVALID_ARG;
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
    // library-owned workspace
    void *ws = nullptr;
    BatchDesc *d_desc = nullptr;
    long long *d_row0 = nullptr, *ub = nullptr, *gsz = nullptr, *goff = nullptr, *bsum = nullptr, *pnnz = nullptr;
    int *prob = nullptr, *cap = nullptr, *nnzc = nullptr, *sym_perm = nullptr, *num_perm = nullptr, *bcount = nullptr;
    unsigned char *sym_bin = nullptr, *num_bin = nullptr;
    unsigned long long *bprod = nullptr;
    RowDesc *rd = nullptr;               // row records of the LDS bins
    int nblk = 0;
    BatchHdr *d_hdr = nullptr, *h_hdr = nullptr;
    int *gkeys = nullptr;
    void *gvals = nullptr;
    long long gcap = 0;                  // slots of gkeys / gvals
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
           g.blocks_per_cu >= 1 && g.blocks_per_cu <= 32;
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
                                       products ? p.bprod : nullptr, nullptr);
    k_bin_scan<<<1, 256, 0, s>>>(p.nblk, p.bcount, products ? p.bprod : nullptr, nullptr, h,
                                 products ? &p.d_hdr->products : nullptr);
    k_scatter<<<p.nblk, 256, 0, s>>>(m, bin_of, p.bcount, h, perm, nullptr, nullptr);
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
    k_bnum_rows<V, LT, S::WPR, S::RPW><<<bgrid(p, blocks_for(p.M, S::RPW)), S::THREADS, 0, s>>>(
        p.d_desc, p.rd, p.d_hdr, LT - kMinLogT, p.ccap, p.ccol, (V *)p.cval, &p.d_hdr->error);
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
        p.d_desc, p.prob, p.d_hdr, p.num_perm, p.goff, p.gcap, p.gkeys, (V *)p.gvals, p.ccap, p.crp, p.ccol,
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
        const size_t vb = p.dtype == SMASH_F32 ? 4 : 8;
        if (p.gkeys) (void)hipFree(p.gkeys);
        if (p.gvals) (void)hipFree(p.gvals);
        p.gkeys = nullptr;
        p.gvals = nullptr;
        p.gcap = 0;
        if (hipMalloc((void **)&p.gkeys, (size_t)need * 4) != hipSuccess ||
            hipMalloc(&p.gvals, (size_t)need * vb) != hipSuccess)
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
    if (p->ws) (void)hipFree(p->ws);
    if (p->gkeys) (void)hipFree(p->gkeys);
    if (p->gvals) (void)hipFree(p->gvals);
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
    const smash_batch_config def{1024, 1, 0, 8};
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
    const size_t need = carve_size({p->desc.size() * sizeof(BatchDesc), ((size_t)count + 1) * 8, (size_t)M * 4,
                                    (size_t)M * 8, (size_t)M * 4, (size_t)M * 4, (size_t)M, (size_t)M,
                                    (size_t)M * 8, (size_t)(M + 1) * 8, (size_t)M * 4, (size_t)M * 4,
                                    (size_t)p->nblk * kNumBins * 4, (size_t)p->nblk * 8, (size_t)(nsb + 1) * 8,
                                    (size_t)std::max(count, 1) * 8, sizeof(BatchHdr), (size_t)M * sizeof(RowDesc)});
    if (hipMalloc(&p->ws, need) != hipSuccess) return bail(fail(c, SMASH_ERR_OUT_OF_MEMORY, "batch workspace"));
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
    if (hipMemcpyAsync(p->d_desc, p->desc.data(), p->desc.size() * sizeof(BatchDesc), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(p->d_row0, p->row0.data(), ((size_t)count + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess)
        return bail(fail(c, SMASH_ERR_HIP, "descriptor upload"));
    if (c->opt[SMASH_OPT_VALIDATE] && count > 0) {
        k_fill_i32<<<1, 256, 0, s>>>((long long)(sizeof(BatchHdr) / sizeof(int)), (int *)p->d_hdr, 0);
        for (int q = 0; q < count && st == SMASH_OK; ++q) {
            st = validate_csr(c, s, A[q], kErrCsrA, &p->d_hdr->error);
            if (st == SMASH_OK) st = validate_csr(c, s, B[q], kErrCsrB, &p->d_hdr->error);
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
            while (fscanf(f, "%255s %d %d %d %d %lf", k, &g.lds_row_max, &g.table_shift, &g.wide_groups,
                          &g.blocks_per_cu, &ms) == 6)
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
                for (int bpc : {4, 16}) {
                    const smash_batch_config g{lrm, sh, wide, bpc};
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
        fprintf(f, "%s %d %d %d %d %.6f\n", key, win.lds_row_max, win.table_shift, win.wide_groups,
                win.blocks_per_cu, top);
        fclose(f);
    }
    return SMASH_OK;
}

}  // extern "C"
