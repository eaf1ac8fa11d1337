// smash_batch.hpp -- kernels of the batched launch: many independent
// products C_p = A_p * B_p run as one pipeline over the concatenated row
// space of all problems.
//
// Global row g of the batch is row g - row0[p] of problem p.  Every kernel
// has a fixed grid (sized from the batch's row count or the machine), reads
// the bin sizes it needs from device memory and loops over its work items,
// so the whole sequence can be captured once in a graph and replayed with no
// host synchronisation: analysis, binning, symbolic per bin, one row-pointer
// scan over the batch (each C_p lands at a device-computed offset of one
// output pool), numeric per bin.  Rows whose bound exceeds the LDS hash
// limit are counted in an LDS bitmap over B's columns and accumulated in LDS
// windows of columns (per-row global tables only for problems wider than
// kWideMaxCols columns).
#pragma once

#include <hip/hip_runtime.h>

#include "smash_kernels.hpp"

namespace smash {

struct BatchDesc {
    const int *Arp, *Acol;
    const void *Aval;
    const int *Brp, *Bcol;
    const void *Bval;
    int rows, cols;
    long long row0;             // first global row of the problem
};

struct BatchHdr {
    BinHdr sym, num;
    unsigned long long products;
    long long nnz_c;            // total entries of all C_p
    long long gneed;            // global table slots of the heavy rows
    int error;
    int wide_queue;             // next heavy row of the windowed numeric kernel
};

// Heavy rows of problems with at most kWideMaxCols columns are counted with
// an LDS bitmap over all columns and accumulated in LDS windows of
// kWideWin columns; wider problems use per-row global tables.
constexpr int kWideMaxCols = 1 << 20;
constexpr int kWideWin = 8192;
constexpr int kWideThreads = 512;

// What an LDS-bin kernel needs of one row, gathered in permutation order by
// k_browdesc so that the bin kernels read one contiguous record per row
// instead of a chain of dependent loads (row id, problem, row pointers,
// C offset).
struct RowDesc {
    int grow;                   // global row
    int prob;                   // problem
    int e0, e1;                 // the row's entries in A_p
    long long rb;               // C offset (numeric only)
    int nc;                     // C entries (numeric only)
    int pad;
};

// Table size class of a row bound: 2^LOGT >= bound << shift slots.
__device__ __forceinline__ int lds_bin_shift(long long bound, int shift)
{
    int lt = ceil_log2(bound << shift);
    return (lt < kMinLogT ? kMinLogT : lt) - kMinLogT;
}

// Per global row: its problem, products ub, bound cap = min(ub, cols), bin
// (empty, LDS by cap << shift, or heavy above lds_row_max) and, for heavy
// rows of problems wider than kWideMaxCols, its global table size.  A wave
// takes 64 consecutive rows, one per lane: the problem of the first by
// binary search over the problems' first rows, the others by stepping
// forward; a lane sums the B-row lengths of its row when the row has at
// most kAnalyzeShort entries, and the whole wave sums each longer row.
constexpr int kAnalyzeShort = 32;

__global__ __launch_bounds__(256) void k_banalyze(long long M, int count, const long long *__restrict__ row0s,
                                                  const BatchDesc *__restrict__ desc, int lds_row_max, int shift,
                                                  int *__restrict__ prob, long long *__restrict__ ub_out,
                                                  int *__restrict__ cap_out, int *__restrict__ nnzc,
                                                  unsigned char *__restrict__ bin_out, long long *__restrict__ gsz)
{
    const int lane = lane_id();
    const long long nw = (long long)gridDim.x * 4;
    for (long long base = ((long long)blockIdx.x * 4 + threadIdx.x / kWave) * kWave; base < M; base += nw * kWave) {
        int lo = 0, hi = count;     // row0s[lo] <= base < row0s[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (row0s[mid] <= base) lo = mid;
            else hi = mid;
        }
        const long long g = base + lane;
        const bool valid = g < M;
        int pr = lo;
        if (valid)
            while (row0s[pr + 1] <= g) ++pr;
        const BatchDesc &d = desc[pr];
        const int row = valid ? (int)(g - d.row0) : 0;
        const int e0 = valid ? d.Arp[row] : 0, e1 = valid ? d.Arp[row + 1] : 0;
        const bool lng = e1 - e0 > kAnalyzeShort;
        long long ub = 0;
        if (!lng) {
            // four entries at a time, so that their loads are in flight together
            int e = e0;
            for (; e + 4 <= e1; e += 4) {
                const int k0 = d.Acol[e], k1 = d.Acol[e + 1], k2 = d.Acol[e + 2], k3 = d.Acol[e + 3];
                ub += (long long)(d.Brp[k0 + 1] - d.Brp[k0]) + (d.Brp[k1 + 1] - d.Brp[k1]) +
                      (d.Brp[k2 + 1] - d.Brp[k2]) + (d.Brp[k3 + 1] - d.Brp[k3]);
            }
            for (; e < e1; ++e) {
                const int k = d.Acol[e];
                ub += d.Brp[k + 1] - d.Brp[k];
            }
        }
        // long rows: the whole wave sums each in turn
        unsigned long long todo = __ballot(valid && lng);
        while (todo) {
            const int src = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const int le0 = __shfl(e0, src, kWave), le1 = __shfl(e1, src, kWave), lp = __shfl(pr, src, kWave);
            const BatchDesc &ld = desc[lp];
            long long part = 0;
            for (int e = le0 + lane; e < le1; e += kWave) {
                const int k = ld.Acol[e];
                part += ld.Brp[k + 1] - ld.Brp[k];
            }
            part = wave_sum(part);
            if (lane == src) ub = part;
        }
        if (valid) {
            const int cap = (int)(ub < d.cols ? ub : d.cols);
            int b = kBinEmpty;
            if (ub > 0) {
                b = cap > lds_row_max ? kBinHeavy : lds_bin_shift(cap, shift);
                if (b >= kLdsBins) b = kBinHeavy;
            }
            prob[g] = pr;
            ub_out[g] = ub;
            cap_out[g] = cap;
            nnzc[g] = 0;
            bin_out[g] = (unsigned char)b;
            gsz[g] = b == kBinHeavy && d.cols > kWideMaxCols ? 1LL << gtable_log2(cap) : 0;
        }
    }
}

// Numeric bins from the exact counts: heavy rows stay heavy, rows without
// entries drop out, LDS rows take the class of their count.
__global__ __launch_bounds__(256) void k_bnum_bins(long long M, int shift, const int *__restrict__ nnzc,
                                                   const unsigned char *__restrict__ sym_bin,
                                                   unsigned char *__restrict__ num_bin)
{
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < M;
         g += (long long)gridDim.x * blockDim.x) {
        const int b = sym_bin[g], nc = nnzc[g];
        num_bin[g] = (unsigned char)(b == kBinHeavy ? kBinHeavy
                                                    : (b == kBinEmpty || nc == 0 ? kBinEmpty : lds_bin_shift(nc, shift)));
    }
}

// Row records of the rows in the LDS bins of one binning (positions
// [0, offset[kLdsBins]) of perm), for k_bsym_rows / k_bnum_rows; with Crp
// non-NULL also their C offsets and counts.
__global__ __launch_bounds__(256) void k_browdesc(const BatchDesc *__restrict__ desc, const int *__restrict__ prob,
                                                  const BinHdr *h, const int *__restrict__ perm,
                                                  const long long *__restrict__ Crp, RowDesc *__restrict__ rd)
{
    const int n = h->offset[kLdsBins];
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        RowDesc o;
        o.grow = perm[r];
        o.prob = prob[o.grow];
        const BatchDesc &d = desc[o.prob];
        const int arow = (int)(o.grow - d.row0);
        o.e0 = d.Arp[arow];
        o.e1 = d.Arp[arow + 1];
        o.rb = Crp ? Crp[o.grow] : 0;
        o.nc = Crp ? (int)(Crp[o.grow + 1] - o.rb) : 0;
        o.pad = 0;
        rd[r] = o;
    }
}

// Symbolic, LDS bin `bin`: RPW rows of WPR waves per work item; the next
// item's row record is loaded while this one is processed.
template <int LOGT, int WPR, int RPW>
__global__ __launch_bounds__(kWave *WPR *RPW) void k_bsym_rows(const BatchDesc *__restrict__ desc,
                                                               const RowDesc *__restrict__ rd, const BinHdr *h,
                                                               int bin, int *__restrict__ nnzc, int *err)
{
    static_assert(RPW == 1 || WPR == 1, "multi-row blocks use one wave per row");
    constexpr int G = WPR * kWave;
    __shared__ int s_keys[RPW][1 << LOGT];
    __shared__ EnumScratch<float, G> s_en[RPW];
    __shared__ int s_cnt[RPW];
    const int cnt = h->count[bin];
    const RowDesc *rows = rd + h->offset[bin];
    const int g = threadIdx.x / kWave / WPR;
    const int gt = threadIdx.x - g * G;
    const int stride = gridDim.x * RPW;
    int base = blockIdx.x * RPW;
    RowDesc cur{};
    if (base + g < cnt) cur = rows[base + g];
    for (; base < cnt; base += stride) {
        const bool active = base + g < cnt;
        RowDesc nxt{};
        if (base + stride + g < cnt) nxt = rows[base + stride + g];
        const BatchDesc &d = desc[active ? cur.prob : 0];
        sym_row<LOGT, WPR>(cur.e0, cur.e1, d.Acol, d.Brp, d.Bcol, active, gt, s_keys[g], s_en[g], &s_cnt[g],
                           &nnzc[active ? cur.grow : 0], err);
        group_sync<WPR>();
        cur = nxt;
    }
}

// Numeric, LDS bin `bin` (row records with C offsets).  Does nothing when
// the output pool is too small (the capacity check has then flagged the
// batch).  HASH as in num_row (0 multiplicative, 1 order-preserving).
template <typename V, int LOGT, int WPR, int RPW, int HASH>
__global__ __launch_bounds__(kWave *WPR *RPW) void k_bnum_rows(const BatchDesc *__restrict__ desc,
                                                               const RowDesc *__restrict__ rd, const BatchHdr *bh,
                                                               int bin, long long ccap, int *__restrict__ Ccol,
                                                               V *__restrict__ Cval, int *err)
{
    static_assert(RPW == 1 || WPR == 1, "multi-row blocks use one wave per row");
    constexpr int T = 1 << LOGT;
    constexpr int G = WPR * kWave;
    __shared__ int s_keys[RPW][T];
    __shared__ double s_vals[RPW][T];
    __shared__ EnumScratch<V, G> s_en[RPW];
    __shared__ int s_scan[RPW][WPR + 1];
    __shared__ int s_maxd[RPW];
    if (bh->nnz_c > ccap) return;
    const int cnt = bh->num.count[bin];
    const RowDesc *rows = rd + bh->num.offset[bin];
    const int g = threadIdx.x / kWave / WPR;
    const int gt = threadIdx.x - g * G;
    const int stride = gridDim.x * RPW;
    int base = blockIdx.x * RPW;
    RowDesc cur{};
    if (base + g < cnt) cur = rows[base + g];
    for (; base < cnt; base += stride) {
        const bool active = base + g < cnt;
        RowDesc nxt{};
        if (base + stride + g < cnt) nxt = rows[base + stride + g];
        const BatchDesc &d = desc[active ? cur.prob : 0];
        num_row<V, LOGT, WPR, HASH>(cur.e0, cur.e1, d.Acol, (const V *)d.Aval, d.Brp, d.Bcol, (const V *)d.Bval,
                                    cur.rb, cur.nc, active, gt, s_keys[g], s_vals[g], s_en[g], s_scan[g], Ccol, Cval,
                                    d.cols, err, &s_maxd[g]);
        group_sync<WPR>();
        cur = nxt;
    }
}

// Symbolic, heavy rows: one block per row, key table at goff[row] in the
// global pool (cleared here; gcap slots in all).
__global__ __launch_bounds__(kGlobalThreads) void k_bsym_global(const BatchDesc *__restrict__ desc,
                                                                const int *__restrict__ prob, const BinHdr *h,
                                                                const int *__restrict__ perm,
                                                                const int *__restrict__ cap,
                                                                const long long *__restrict__ goff, long long gcap,
                                                                int *gkeys, int *__restrict__ nnzc, int *err)
{
    __shared__ EnumScratch<float, kGlobalThreads> S;
    __shared__ int s_cnt;
    const int cnt = h->count[kBinHeavy];
    const int *rows = perm + h->offset[kBinHeavy];
    for (int r = blockIdx.x; r < cnt; r += gridDim.x) {
        const int grow = rows[r];
        const BatchDesc &d = desc[prob[grow]];
        if (d.cols <= kWideMaxCols) continue;
        const long long off = goff[grow];
        const int T = 1 << gtable_log2(cap[grow]);
        if (off + T > gcap) {
            if (threadIdx.x == 0) atomicOr(err, kErrCapacity);
            continue;
        }
        int *keys = gkeys + off;
        for (int t = threadIdx.x; t < T; t += kGlobalThreads) keys[t] = kEmpty;
        __threadfence();
        __syncthreads();
        sym_global_row(d.Arp, d.Acol, d.Brp, d.Bcol, (int)(grow - d.row0), cap[grow], keys, S, &s_cnt, &nnzc[grow],
                       err);
        __syncthreads();
    }
}

// Numeric, heavy rows: one block per row (dynamic LDS: the rank bitmap).
template <typename V>
__global__ __launch_bounds__(kGlobalThreads) void k_bnum_global(const BatchDesc *__restrict__ desc,
                                                                const int *__restrict__ prob, const BatchHdr *bh,
                                                                const int *__restrict__ perm,
                                                                const long long *__restrict__ goff, long long gcap,
                                                                int *gkeys, double *gvals, int *gtouch, long long ccap,
                                                                const long long *__restrict__ Crp,
                                                                int *__restrict__ Ccol, V *__restrict__ Cval, int *err)
{
    extern __shared__ unsigned s_bm[];
    __shared__ GlobalNumLds<V> L;
    if (bh->nnz_c > ccap) return;
    const int cnt = bh->num.count[kBinHeavy];
    const int *rows = perm + bh->num.offset[kBinHeavy];
    for (int r = blockIdx.x; r < cnt; r += gridDim.x) {
        const int grow = rows[r];
        const BatchDesc &d = desc[prob[grow]];
        if (d.cols <= kWideMaxCols) continue;
        const long long off = goff[grow];
        const int nc = (int)(Crp[grow + 1] - Crp[grow]);
        if (off + (1LL << gtable_log2(nc)) > gcap) {
            if (threadIdx.x == 0) atomicOr(err, kErrCapacity);
            continue;
        }
        num_global_row<V>(d.Arp, d.Acol, (const V *)d.Aval, d.Brp, d.Bcol, (const V *)d.Bval, (int)(grow - d.row0),
                          grow, d.cols, gkeys + off, gvals + off, gtouch + off, L, s_bm, Crp, Ccol, Cval, err);
        __syncthreads();
    }
}

// Symbolic, heavy rows of problems with at most kWideMaxCols columns: one
// block per row sets one bit per column of the row in an LDS bitmap over all
// of B's columns (dynamic LDS, ceil(cols / 32) words) and counts the bits.
__global__ __launch_bounds__(kWideThreads) void k_bsym_wide(const BatchDesc *__restrict__ desc,
                                                            const int *__restrict__ prob, const BinHdr *h,
                                                            const int *__restrict__ perm, int *__restrict__ nnzc)
{
    extern __shared__ unsigned s_bmw[];
    __shared__ EnumScratch<float, kWideThreads> S;
    __shared__ int s_cnt;
    const int cnt = h->count[kBinHeavy];
    const int *rows = perm + h->offset[kBinHeavy];
    const int gt = threadIdx.x;
    for (int r = blockIdx.x; r < cnt; r += gridDim.x) {
        const int grow = rows[r];
        const BatchDesc &d = desc[prob[grow]];
        if (d.cols > kWideMaxCols) continue;
        const int nw = (d.cols + 31) >> 5;
        const int *Acol = d.Acol, *Brp = d.Brp;
        const int arow = (int)(grow - d.row0);
        for (int t = gt; t < nw; t += kWideThreads) s_bmw[t] = 0u;
        if (gt == 0) s_cnt = 0;
        __syncthreads();
        group_products<float, false, kWideThreads, 2>(
            d.Arp[arow], d.Arp[arow + 1], gt, S, d.Bcol, (const float *)nullptr,
            [&](int e, int &bs, int &bl, float &) {
                const int k = Acol[e];
                bs = Brp[k];
                bl = Brp[k + 1] - bs;
            },
            [&](int j) {
                const unsigned bit = 1u << (j & 31);
                if (!(s_bmw[j >> 5] & bit)) atomicOr(&s_bmw[j >> 5], bit);
            });
        __syncthreads();
        int c = 0;
        for (int t = gt; t < nw; t += kWideThreads) c += __popc(s_bmw[t]);
        c = wave_sum(c);
        if (lane_id() == 0 && c) atomicAdd(&s_cnt, c);
        __syncthreads();
        if (gt == 0) nnzc[grow] = s_cnt;
    }
}

// Numeric, heavy rows of problems with at most kWideMaxCols columns: one
// block per row takes B's columns in windows of kWideWin; in each window the
// row's products with columns inside it are added into an LDS array of
// doubles indexed by column (occupancy marked by the -0.0 start value, as in
// the dense chunks of single products), and each wave ranks its share of the
// window with ballots and stores its entries in column order through its own
// slots (dynamic LDS: the kWideWin doubles).  Each window enumerates only the B entries inside
// it: a row with at most kWideThreads A entries keeps, per thread, a cursor
// into its B row that the windows advance (one search per window); longer
// rows search both window bounds in every B row they visit.
template <typename V>
__global__ __launch_bounds__(kWideThreads) void k_bnum_wide(const BatchDesc *__restrict__ desc,
                                                            const int *__restrict__ prob, const BatchHdr *bh,
                                                            const int *__restrict__ perm, long long ccap,
                                                            const long long *__restrict__ Crp, int *__restrict__ Ccol,
                                                            V *__restrict__ Cval, int *err, int *queue)
{
    constexpr int NW = kWideThreads / kWave;
    constexpr int CPW = kWideWin / NW;                  // columns ranked by each wave
    constexpr int ROUNDS = CPW / kWave;
    extern __shared__ __align__(16) unsigned char s_raw[];
    double *acc = (double *)s_raw;                      // [kWideWin]
    __shared__ EnumScratch<V, kWideThreads> S;
    __shared__ int s_wt[NW];
    __shared__ int s_r;
    if (bh->nnz_c > ccap) return;
    const int cnt = bh->num.count[kBinHeavy];
    const int *rows = perm + bh->num.offset[kBinHeavy];
    const int gt = threadIdx.x, lane = lane_id(), wg = gt / kWave;
    // heavy rows from a queue (one atomic per row): long and short rows
    // balance across the persistent blocks
    for (;;) {
        __syncthreads();                                // the previous row is done with s_r and the window
        if (gt == 0) s_r = atomicAdd(queue, 1);
        __syncthreads();
        const int r = s_r;
        if (r >= cnt) break;
        const int grow = rows[r];
        const BatchDesc &d = desc[prob[grow]];
        if (d.cols > kWideMaxCols) continue;
        const int *Acol = d.Acol, *Brp = d.Brp;
        const V *Aval = (const V *)d.Aval;
        const int arow = (int)(grow - d.row0);
        const long long rb = Crp[grow];
        const int nc = (int)(Crp[grow + 1] - rb);
        const int e0 = d.Arp[arow], e1 = d.Arp[arow + 1];
        const bool single = e1 - e0 <= kWideThreads;       // one A entry per thread at most
        int cur = 0, bend = 0;                             // this thread's B row: next entry, end
        if (single && gt < e1 - e0) {
            const int k = Acol[e0 + gt];
            cur = Brp[k];
            bend = Brp[k + 1];
        }
        int done = 0;
        for (int lo = 0; lo < d.cols; lo += kWideWin) {
            const int hi = lo + kWideWin;
            const int nxt = single && gt < e1 - e0 ? lower_bound_col(d.Bcol, cur, bend, hi) : 0;
            for (int t = gt; t < kWideWin; t += kWideThreads) acc[t] = -0.0;
            __syncthreads();
            group_products<V, true, kWideThreads, 2>(
                e0, e1, gt, S, d.Bcol, (const V *)d.Bval,
                [&](int e, int &bs, int &bl, V &a) {
                    if (single) {                          // e is this thread's entry
                        bs = cur;
                        bl = nxt - cur;
                    } else {
                        const int k = Acol[e];
                        const int b1 = Brp[k + 1];
                        bs = lower_bound_col(d.Bcol, Brp[k], b1, lo);
                        bl = lower_bound_col(d.Bcol, bs, b1, hi) - bs;
                    }
                    a = Aval[e];
                },
                [&](int j, double p) {
                    const unsigned jl = (unsigned)(j - lo);
                    if (jl < (unsigned)kWideWin) atomicAdd(&acc[jl], p + 0.0);
                });
            cur = nxt;
            __syncthreads();
            double vr[ROUNDS];
            unsigned long long msk[ROUNDS];
            int wcount = 0;
#pragma unroll
            for (int q = 0; q < ROUNDS; ++q) {
                const int jl = wg * CPW + q * kWave + lane;
                vr[q] = acc[jl];
                msk[q] = wave_ballot(reached(vr[q]));
                wcount += __popcll(msk[q]);
            }
            if (lane == 0) s_wt[wg] = wcount;
            __syncthreads();
            int run = done, tot = 0;
            for (int w = 0; w < NW; ++w) {
                const int t = s_wt[w];
                if (w < wg) run += t;
                tot += t;
            }
            const int n = wcount < nc - run ? wcount : (nc - run > 0 ? nc - run : 0);
            wave_store_ranked<V, ROUNDS>(vr, msk, acc + wg * CPW, lo + wg * CPW, rb + run, n, Ccol, Cval);
            done += tot;
            __syncthreads();
        }
        if (gt == 0 && done != nc) atomicOr(err, kErrCount);
    }
}

// Flags a batch whose entries exceed the output pool.
__global__ void k_bcheck(BatchHdr *bh, long long ccap)
{
    if (threadIdx.x == 0 && bh->nnz_c > ccap) atomicOr(&bh->error, kErrCapacity);
}

// Entries of each problem: nnz[p] = Crp[row0[p + 1]] - Crp[row0[p]].
__global__ __launch_bounds__(256) void k_bproblem_nnz(int count, const long long *__restrict__ row0s,
                                                      const long long *__restrict__ Crp, long long *__restrict__ nnz)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < count) nnz[p] = Crp[row0s[p + 1]] - Crp[row0s[p]];
}

}  // namespace smash
