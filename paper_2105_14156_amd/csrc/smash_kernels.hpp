// smash_kernels.hpp -- gfx950 kernels of the row-wise hash SpGEMM C = A * B.
//
// Method (SMASH thesis, arXiv 2105.14156): the row-wise product of the
// Background chapter (eq. "row_wise"), where each output row's partial
// products are merged in an on-chip hash table as they are generated, with an
// atomic compare-and-swap claiming empty slots and an atomic fetch-and-add
// merging values (SMASH Kernels chapter, "Hashing Phase").  The output is
// sized from per-row product counts (Window Distribution Phase) refined by an
// exact symbolic pass, and written back as sorted CSR (Write-back Phase).
//
// MI355X mapping (not the PIUMA design of the paper):
//   * one 64-lane wavefront, or a group of wavefronts, owns one output row
//     and its LDS table; rows are binned by table size so every bin launches
//     a workgroup shape that fits its rows (the paper's windows sized to the
//     scratchpad);
//   * the products of a row are enumerated "flat": a wave loads 64 entries
//     of A's row, prefix-sums the lengths of the B rows they select, and
//     every lane takes one product per step, so a long B row and many short
//     ones keep all 64 lanes busy (the paper splits rows between two
//     threads for the same reason, "SMASH Version 2: Tokenization");
//   * slots come from a multiplicative (Fibonacci) hash of the column, which
//     spreads clustered columns like the paper's low-order-bit hash of
//     version 2, with +1 linear probing;
//   * rows whose output does not fit an LDS table take the heavy-row path:
//     either column windows accumulated densely in LDS (the paper's per-row
//     dense/sparse decision of the Window Distribution Phase), or a hash
//     table in global memory (version 3, "Fragmenting Memory").
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smash {

constexpr int kWave = 64;
constexpr int kEmpty = -1;              // empty-slot tag (Algorithm "SMASH SETUP": EMPTY = -1)
constexpr int kMinLogT = 6;             // smallest LDS table: 64 slots
constexpr int kMaxLogT = 13;            // largest LDS table: 8192 slots
constexpr int kLdsBins = kMaxLogT - kMinLogT + 1;
constexpr int kBinHeavy = kLdsBins;
constexpr int kBinEmpty = kLdsBins + 1;
constexpr int kNumBins = kLdsBins + 2;
constexpr int kChunkCols = 8192;        // column granularity of heavy-row counts
constexpr int kChunkWords = kChunkCols / 32;
constexpr int kSymWindowBits = 1 << 20; // symbolic heavy-row bitmap window (128 KiB)
constexpr int kHeavyThreads = 1024;

enum : int {
    kErrProbe = 1,      // a hash table ran out of slots (inconsistent sizes)
    kErrCsrA = 2,       // A violates the CSR preconditions
    kErrCsrB = 4,       // B violates the CSR preconditions
    kErrCount = 8,      // numeric found a row count different from C_row_ptr
};

struct BinHdr {
    int count[kNumBins];      // rows per bin
    int offset[kNumBins + 1]; // exclusive offsets of the bins in the row permutation
    int cursor[kNumBins];     // scatter cursors
};

struct DevHdr {
    unsigned long long products;       // sum over rows of products
    unsigned long long gneed[2];       // global-hash slots needed: [0] symbolic, [1] numeric
    unsigned long long gcursor[2];     // global-hash slots handed out so far
    long long nnz_c;
    BinHdr sym, num;
    int error;
    int heavy_windows;
    int pad[2];
};

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Orders LDS accesses of one wavefront (lanes execute in lockstep; the fence
// keeps the compiler from moving LDS reads above earlier writes).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <int WAVES>
__device__ __forceinline__ void group_sync()
{
    if constexpr (WAVES == 1) wave_sync();
    else __syncthreads();
}

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ __forceinline__ int ceil_log2(long long x)
{
    return x <= 1 ? 0 : 64 - __clzll((unsigned long long)(x - 1));
}

// Fibonacci hashing of a column index onto 2^logT slots.
__device__ __forceinline__ unsigned slot_of(int key, int logT)
{
    return ((unsigned)key * 2654435769u) >> (32 - logT);
}

// log2 of the global hash table size of a heavy row with at most n keys
// (load factor at most one half).
__device__ __forceinline__ int gtable_log2(long long n)
{
    return ceil_log2(2LL * (n > 1 ? n : 1));
}

// Bin of a row for the symbolic phase, from its product count ub and output
// bound cap = min(ub, cols).
__device__ __forceinline__ int sym_bin(long long ub, int cap, int lds_row_max)
{
    if (ub == 0) return kBinEmpty;
    if (cap > lds_row_max) return kBinHeavy;
    int lt = ceil_log2(2LL * cap);
    return (lt < kMinLogT ? kMinLogT : lt) - kMinLogT;
}

// Bin of a row for the numeric phase, from its exact output count.
__device__ __forceinline__ int num_bin(int nc, bool heavy)
{
    if (heavy) return kBinHeavy;
    if (nc == 0) return kBinEmpty;
    int lt = ceil_log2(2LL * nc);
    return (lt < kMinLogT ? kMinLogT : lt) - kMinLogT;
}

// Block-wide exclusive scan of one value per thread (all threads call it).
template <typename T, int THREADS>
__device__ __forceinline__ T block_excl_scan(T v, T *s_tmp /* THREADS/64 + 1 */, T &total)
{
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    T incl = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T t = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += t;
    }
    if (lane == kWave - 1) s_tmp[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < THREADS / kWave; ++w) { T t = s_tmp[w]; s_tmp[w] = run; run += t; }
        s_tmp[THREADS / kWave] = run;
    }
    __syncthreads();
    T res = s_tmp[wave] + incl - v;
    total = s_tmp[THREADS / kWave];
    __syncthreads();
    return res;
}

// ----------------------------------------------------- product enumeration
//
// Calls sink(j, a * b) (or sink(j) without values) for every product of the
// A entries [e0, e1) of one row, restricted to the B ranges returned by
// get(e, &bstart, &blen, &a).  The waves of a group stride over chunks of 64
// A entries; within a chunk each lane takes products q = lane, lane + 64, ...
// of the concatenated B ranges and finds its A entry by a 6-step search of
// the chunk's inclusive length prefix (kept in LDS, one 64-entry slice per
// wave).
template <typename V, bool WITH_VAL, typename Get, typename Sink>
__device__ __forceinline__ void wave_products(int e0, int e1, int wave_in_group, int waves_in_group,
                                              int *s_incl, int *s_bs, V *s_a,
                                              const int *__restrict__ Bcol, const V *__restrict__ Bval,
                                              Get get, Sink sink)
{
    const int lane = lane_id();
    for (int base = e0 + wave_in_group * kWave; base < e1; base += waves_in_group * kWave) {
        const int e = base + lane;
        int bs = 0, bl = 0;
        V a = V(0);
        if (e < e1) get(e, bs, bl, a);
        const int incl = wave_incl_scan(bl);
        const int total = __shfl(incl, kWave - 1, kWave);
        s_incl[lane] = incl;
        s_bs[lane] = bs;
        if constexpr (WITH_VAL) s_a[lane] = a;
        wave_sync();
        for (int q = lane; q < total; q += kWave) {
            int src = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1)
                if (s_incl[src + step - 1] <= q) src += step;
            const int excl = src ? s_incl[src - 1] : 0;
            const int pos = s_bs[src] + (q - excl);
            const int j = Bcol[pos];
            if constexpr (WITH_VAL) sink(j, s_a[src] * Bval[pos]);
            else sink(j);
        }
        wave_sync();
    }
}

// ------------------------------------------------------------ LDS hashing

// Claims the slot of `key` in an LDS key table; returns 1 if the key was new.
__device__ __forceinline__ int lds_insert_key(int *keys, int logT, int key, int *err)
{
    const unsigned mask = (1u << logT) - 1;
    unsigned h = slot_of(key, logT);
    for (unsigned probe = 0; probe <= mask; ++probe) {
        int cur = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == key) return 0;
        if (cur == kEmpty) {
            int old = atomicCAS(&keys[h], kEmpty, key);
            if (old == kEmpty) return 1;
            if (old == key) return 0;
        }
        h = (h + 1) & mask;
    }
    atomicOr(err, kErrProbe);
    return 0;
}

// Claims or finds the slot of `key` and adds `p` to its value.
template <typename V>
__device__ __forceinline__ void lds_insert_add(int *keys, V *vals, int logT, int key, V p, int *err)
{
    const unsigned mask = (1u << logT) - 1;
    unsigned h = slot_of(key, logT);
    for (unsigned probe = 0; probe <= mask; ++probe) {
        int cur = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == kEmpty) {
            int old = atomicCAS(&keys[h], kEmpty, key);
            cur = old == kEmpty ? key : old;
        }
        if (cur == key) {
            atomicAdd(&vals[h], p);
            return;
        }
        h = (h + 1) & mask;
    }
    atomicOr(err, kErrProbe);
}

// --------------------------------------------------------- analysis & bins

// Row analysis (step a1): products ub_i = sum_k nnz(B_k) over row i of A, the
// output bound cap_i = min(ub_i, cols), the symbolic bin of the row, and the
// totals.  One wave per row, four rows per block.
__global__ __launch_bounds__(256) void k_analyze(int m, int ncols, int lds_row_max,
                                                 const int *__restrict__ Arp, const int *__restrict__ Acol,
                                                 const int *__restrict__ Brp, long long *__restrict__ ub_out,
                                                 int *__restrict__ cap_out, int *__restrict__ nnzc,
                                                 unsigned char *__restrict__ bin_out, DevHdr *hdr)
{
    __shared__ int s_hist[kNumBins];
    __shared__ unsigned long long s_prod, s_gslots;
    if (threadIdx.x < kNumBins) s_hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) { s_prod = 0; s_gslots = 0; }
    __syncthreads();
    const int lane = lane_id();
    const int row = blockIdx.x * 4 + threadIdx.x / kWave;
    if (row < m) {
        const int e0 = Arp[row], e1 = Arp[row + 1];
        long long ub = 0;
        for (int e = e0 + lane; e < e1; e += kWave) {
            const int k = Acol[e];
            ub += Brp[k + 1] - Brp[k];
        }
        ub = wave_sum(ub);
        if (lane == 0) {
            const int cap = (int)(ub < ncols ? ub : ncols);
            const int b = sym_bin(ub, cap, lds_row_max);
            ub_out[row] = ub;
            cap_out[row] = cap;
            nnzc[row] = 0;
            bin_out[row] = (unsigned char)b;
            atomicAdd(&s_hist[b], 1);
            atomicAdd(&s_prod, (unsigned long long)ub);
            if (b == kBinHeavy) atomicAdd(&s_gslots, 1ull << gtable_log2(cap));
        }
    }
    __syncthreads();
    if (threadIdx.x < kNumBins && s_hist[threadIdx.x]) atomicAdd(&hdr->sym.count[threadIdx.x], s_hist[threadIdx.x]);
    if (threadIdx.x == 0) {
        if (s_prod) atomicAdd(&hdr->products, s_prod);
        if (s_gslots) atomicAdd(&hdr->gneed[0], s_gslots);
    }
}

// Exclusive offsets of the bins and scatter cursors (one thread).
__global__ void k_bin_offsets(BinHdr *h)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int run = 0;
    for (int b = 0; b < kNumBins; ++b) {
        h->offset[b] = run;
        h->cursor[b] = run;
        run += h->count[b];
    }
    h->offset[kNumBins] = run;
}

// Groups row ids by bin (empty rows are left out).  Rows of the heavy bin
// that use the global hash table also get their table's slot offset.
__global__ __launch_bounds__(256) void k_scatter(int m, const unsigned char *__restrict__ bin_of,
                                                 BinHdr *h, int *__restrict__ perm,
                                                 const int *__restrict__ heavy_size /* nullable */,
                                                 unsigned long long *gcursor, long long *__restrict__ goff)
{
    __shared__ int s_cnt[kNumBins], s_base[kNumBins];
    __shared__ unsigned long long s_gsum, s_gbase;
    if (threadIdx.x < kNumBins) s_cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_gsum = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = i < m ? (int)bin_of[i] : -1;
    const int local = b >= 0 ? atomicAdd(&s_cnt[b], 1) : 0;
    unsigned long long gsz = 0, gloc = 0;
    if (b == kBinHeavy && heavy_size) {
        gsz = 1ull << gtable_log2(heavy_size[i]);
        gloc = atomicAdd(&s_gsum, gsz);
    }
    __syncthreads();
    if (threadIdx.x < kNumBins && threadIdx.x != kBinEmpty && s_cnt[threadIdx.x])
        s_base[threadIdx.x] = atomicAdd(&h->cursor[threadIdx.x], s_cnt[threadIdx.x]);
    if (threadIdx.x == 0 && heavy_size && s_gsum) s_gbase = atomicAdd(gcursor, s_gsum);
    __syncthreads();
    if (b >= 0 && b != kBinEmpty) {
        const int pos = s_base[b] + local;
        perm[pos] = i;
        if (b == kBinHeavy && heavy_size) goff[pos - h->offset[kBinHeavy]] = (long long)(s_gbase + gloc);
    }
}

// Numeric bins from the exact row counts; heavy rows stay heavy.  Also sums
// the global-hash slots the heavy rows need in global mode.
__global__ __launch_bounds__(256) void k_num_bins(int m, const int *__restrict__ nnzc,
                                                  const unsigned char *__restrict__ sym_bin_of,
                                                  unsigned char *__restrict__ bin_out, DevHdr *hdr)
{
    __shared__ int s_hist[kNumBins];
    __shared__ unsigned long long s_gslots;
    if (threadIdx.x < kNumBins) s_hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_gslots = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) {
        const bool heavy = sym_bin_of[i] == kBinHeavy;
        const int b = num_bin(nnzc[i], heavy);
        bin_out[i] = (unsigned char)b;
        atomicAdd(&s_hist[b], 1);
        if (heavy) atomicAdd(&s_gslots, 1ull << gtable_log2(nnzc[i]));
    }
    __syncthreads();
    if (threadIdx.x < kNumBins && s_hist[threadIdx.x]) atomicAdd(&hdr->num.count[threadIdx.x], s_hist[threadIdx.x]);
    if (threadIdx.x == 0 && s_gslots) atomicAdd(&hdr->gneed[1], s_gslots);
}

// --------------------------------------------------------------- validation

// Checks the CSR preconditions of one matrix; sets `flag` in *err on failure.
__global__ __launch_bounds__(256) void k_validate(int rows, int cols, long long nnz, const int *__restrict__ rp,
                                                  const int *__restrict__ ci, int flag, int *err)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (i == 0 && (rp[0] != 0 || (long long)rp[rows] != nnz)) bad = true;
    if (i < rows) {
        const int a = rp[i], b = rp[i + 1];
        if (b < a || a < 0 || (long long)b > nnz) bad = true;
        else {
            for (int p = a; p < b; ++p) {
                const int c = ci[p];
                if (c < 0 || c >= cols || (p > a && c <= ci[p - 1])) { bad = true; break; }
            }
        }
    }
    if (bad) atomicOr(err, flag);
}

// ------------------------------------------------------- symbolic, LDS hash

// One row per group of WPR waves (RPW groups per block; RPW > 1 only with
// WPR = 1).  Counts the distinct columns of each row with an LDS key table
// of 2^LOGT slots (step a3).
template <int LOGT, int WPR, int RPW>
__global__ __launch_bounds__(kWave *WPR *RPW) void k_sym_lds(const int *__restrict__ Arp, const int *__restrict__ Acol,
                                                             const int *__restrict__ Brp, const int *__restrict__ Bcol,
                                                             const int *__restrict__ rows, int nrows,
                                                             int *__restrict__ nnzc, int *err)
{
    static_assert(RPW == 1 || WPR == 1, "multi-row blocks use one wave per row");
    constexpr int T = 1 << LOGT;
    __shared__ int s_keys[RPW][T];
    __shared__ int s_incl[RPW * WPR][kWave];
    __shared__ int s_bs[RPW * WPR][kWave];
    __shared__ int s_cnt[RPW];
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const int g = wave / WPR, wg = wave % WPR;
    const int r = blockIdx.x * RPW + g;
    const bool active = r < nrows;
    const int row = active ? rows[r] : 0;
    for (int t = wg * kWave + lane; t < T; t += WPR * kWave) s_keys[g][t] = kEmpty;
    if (wg == 0 && lane == 0) s_cnt[g] = 0;
    group_sync<WPR>();
    int mine = 0;
    if (active) {
        int *keys = s_keys[g];
        wave_products<float, false>(
            Arp[row], Arp[row + 1], wg, WPR, s_incl[wave], s_bs[wave], (float *)nullptr, Bcol, (const float *)nullptr,
            [&](int e, int &bs, int &bl, float &) {
                const int k = Acol[e];
                bs = Brp[k];
                bl = Brp[k + 1] - bs;
            },
            [&](int j) { mine += lds_insert_key(keys, LOGT, j, err); });
    }
    mine = wave_sum(mine);
    if (lane == 0 && mine) atomicAdd(&s_cnt[g], mine);
    group_sync<WPR>();
    if (active && wg == 0 && lane == 0) nnzc[row] = s_cnt[g];
}

// -------------------------------------------------------- numeric, LDS hash

// Key-value bitonic sort of n2 (a power of two) LDS entries by a group of
// G threads whose index in the group is gt.
template <typename V, int WPR>
__device__ __forceinline__ void group_bitonic(int *keys, V *vals, int n2, int gt)
{
    constexpr int G = WPR * kWave;
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int p = gt; p < (n2 >> 1); p += G) {
                const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
                const int l = i + j;
                const bool up = (i & k) == 0;
                const int ki = keys[i], kl = keys[l];
                if ((ki > kl) == up) {
                    keys[i] = kl;
                    keys[l] = ki;
                    const V vi = vals[i];
                    vals[i] = vals[l];
                    vals[l] = vi;
                }
            }
            group_sync<WPR>();
        }
    }
}

// Numeric phase of light rows (steps a5 and a7): products merged in an LDS
// tag/value table of 2^LOGT slots, then the occupied slots compacted,
// sorted by column and written at the row's offset in C.
template <typename V, int LOGT, int WPR, int RPW>
__global__ __launch_bounds__(kWave *WPR *RPW) void k_num_lds(
    const int *__restrict__ Arp, const int *__restrict__ Acol, const V *__restrict__ Aval,
    const int *__restrict__ Brp, const int *__restrict__ Bcol, const V *__restrict__ Bval,
    const int *__restrict__ rows, int nrows, const long long *__restrict__ Crp, int *__restrict__ Ccol,
    V *__restrict__ Cval, int *err)
{
    static_assert(RPW == 1 || WPR == 1, "multi-row blocks use one wave per row");
    constexpr int T = 1 << LOGT;
    constexpr int G = WPR * kWave;
    constexpr int SPT = T / G;          // slots per thread in the compaction
    static_assert(SPT >= 1, "table smaller than its group");
    __shared__ int s_keys[RPW][T];
    __shared__ V s_vals[RPW][T];
    __shared__ int s_incl[RPW * WPR][kWave];
    __shared__ int s_bs[RPW * WPR][kWave];
    __shared__ V s_a[RPW * WPR][kWave];
    __shared__ int s_scan[RPW][WPR + 1];
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const int g = wave / WPR, wg = wave % WPR;
    const int gt = wg * kWave + lane;
    const int r = blockIdx.x * RPW + g;
    const bool active = r < nrows;
    const int row = active ? rows[r] : 0;
    int *keys = s_keys[g];
    V *vals = s_vals[g];
    for (int t = gt; t < T; t += G) {
        keys[t] = kEmpty;
        vals[t] = V(0);
    }
    group_sync<WPR>();
    if (active) {
        wave_products<V, true>(
            Arp[row], Arp[row + 1], wg, WPR, s_incl[wave], s_bs[wave], s_a[wave], Bcol, Bval,
            [&](int e, int &bs, int &bl, V &a) {
                const int k = Acol[e];
                bs = Brp[k];
                bl = Brp[k + 1] - bs;
                a = Aval[e];
            },
            [&](int j, V p) { lds_insert_add(keys, vals, LOGT, j, p, err); });
    }
    group_sync<WPR>();
    // compaction of the occupied slots to the front of the table
    int kr[SPT];
    V vr[SPT];
    int cnt = 0;
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        kr[s] = keys[gt * SPT + s];
        vr[s] = vals[gt * SPT + s];
        cnt += kr[s] != kEmpty;
    }
    int incl = wave_incl_scan(cnt);
    if (lane == kWave - 1) s_scan[g][wg] = incl;
    group_sync<WPR>();
    int wbase = 0, total = 0;
    for (int w = 0; w < WPR; ++w) {
        const int t = s_scan[g][w];
        if (w < wg) wbase += t;
        total += t;
    }
    int pos = wbase + incl - cnt;
    group_sync<WPR>();
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        if (kr[s] != kEmpty) {
            keys[pos] = kr[s];
            vals[pos] = vr[s];
            ++pos;
        }
    }
    const int n2 = total <= 1 ? 1 : (1 << ceil_log2(total));
    for (int t = total + gt; t < n2; t += G) keys[t] = 0x7fffffff;
    group_sync<WPR>();
    group_bitonic<V, WPR>(keys, vals, n2, gt);
    if (active) {
        const long long rb = Crp[row];
        const int nc = (int)(Crp[row + 1] - rb);
        if (gt == 0 && nc != total) atomicOr(err, kErrCount);
        const int nw = total < nc ? total : nc;
        for (int t = gt; t < nw; t += G) {
            Ccol[rb + t] = keys[t];
            Cval[rb + t] = vals[t];
        }
    }
}

// ---------------------------------------------------------------- row scan

// C_row_ptr = exclusive prefix of the row counts, in three passes over
// blocks of kScanItems rows.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanItems = kScanThreads * kScanPer;

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(int m, const int *__restrict__ cnt,
                                                              long long *__restrict__ bsum)
{
    __shared__ long long s_tmp[kScanThreads / kWave + 1];
    const long long base = (long long)blockIdx.x * kScanItems + threadIdx.x * kScanPer;
    long long s = 0;
#pragma unroll
    for (int t = 0; t < kScanPer; ++t)
        if (base + t < m) s += cnt[base + t];
    long long total;
    block_excl_scan<long long, kScanThreads>(s, s_tmp, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(int nb, long long *__restrict__ bsum,
                                                           long long *__restrict__ total_out)
{
    __shared__ long long s_tmp[kScanThreads / kWave + 1];
    __shared__ long long s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int b = b0 + threadIdx.x;
        const long long v = b < nb ? bsum[b] : 0;
        long long tot;
        const long long ex = block_excl_scan<long long, kScanThreads>(v, s_tmp, tot);
        const long long carry = s_carry;
        if (b < nb) bsum[b] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total_out = s_carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int m, const int *__restrict__ cnt,
                                                             const long long *__restrict__ boff,
                                                             const long long *__restrict__ total,
                                                             long long *__restrict__ out)
{
    __shared__ long long s_tmp[kScanThreads / kWave + 1];
    const long long base = (long long)blockIdx.x * kScanItems + threadIdx.x * kScanPer;
    int v[kScanPer];
    long long s = 0;
#pragma unroll
    for (int t = 0; t < kScanPer; ++t) {
        v[t] = base + t < m ? cnt[base + t] : 0;
        s += v[t];
    }
    long long tot;
    long long run = block_excl_scan<long long, kScanThreads>(s, s_tmp, tot) + boff[blockIdx.x];
#pragma unroll
    for (int t = 0; t < kScanPer; ++t) {
        if (base + t < m) out[base + t] = run;
        run += v[t];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[m] = *total;
}

// ------------------------------------------------- heavy rows: windowed path

// lower_bound of `x` in the ascending columns Bcol[lo, hi).
__device__ __forceinline__ int lower_bound_col(const int *__restrict__ Bcol, int lo, int hi, int x)
{
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (Bcol[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Symbolic phase of heavy rows: one block per row marks the row's columns in
// an LDS bitmap over windows of kSymWindowBits columns and records the
// number of columns in every kChunkCols-wide chunk (wcnt) and in the row.
__global__ __launch_bounds__(kHeavyThreads) void k_sym_heavy(
    const int *__restrict__ Arp, const int *__restrict__ Acol, const int *__restrict__ Brp,
    const int *__restrict__ Bcol, const int *__restrict__ rows, int ncols, int nchunks,
    int *__restrict__ wcnt, int *__restrict__ nnzc, int *err)
{
    extern __shared__ unsigned s_dyn[];
    constexpr int NW = kHeavyThreads / kWave;
    unsigned *bm = s_dyn;                                           // window bitmap
    const int wbits = ncols < kSymWindowBits ? ((ncols + 31) & ~31) : kSymWindowBits;
    const int words = wbits / 32;
    int *s_incl = (int *)(bm + words);                              // [NW][64]
    int *s_bs = s_incl + NW * kWave;                                // [NW][64]
    __shared__ int s_row_total;
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const int row = rows[blockIdx.x];
    const int e0 = Arp[row], e1 = Arp[row + 1];
    const int nwin = (ncols + kSymWindowBits - 1) / kSymWindowBits;
    if (threadIdx.x == 0) s_row_total = 0;
    for (int w = 0; w < nwin; ++w) {
        const int lo = w * kSymWindowBits;
        const int hi = lo + wbits < ncols ? lo + wbits : ncols;
        for (int t = threadIdx.x; t < words; t += kHeavyThreads) bm[t] = 0u;
        __syncthreads();
        wave_products<float, false>(
            e0, e1, wave, NW, s_incl + wave * kWave, s_bs + wave * kWave, (float *)nullptr, Bcol,
            (const float *)nullptr,
            [&](int e, int &bs, int &bl, float &) {
                const int k = Acol[e];
                int b0 = Brp[k], b1 = Brp[k + 1];
                if (nwin > 1) {
                    b0 = lower_bound_col(Bcol, b0, b1, lo);
                    b1 = lower_bound_col(Bcol, b0, b1, hi);
                }
                bs = b0;
                bl = b1 - b0;
            },
            [&](int j) {
                const int jl = j - lo;
                atomicOr(&bm[jl >> 5], 1u << (jl & 31));
            });
        __syncthreads();
        // per-chunk counts: kChunkWords words per chunk
        const int first_chunk = lo / kChunkCols;
        const int wchunks = (words + kChunkWords - 1) / kChunkWords;
        int local = 0;
        for (int c = wave; c < wchunks; c += NW) {
            int pc = 0;
            for (int t = lane; t < kChunkWords; t += kWave) {
                const int wd = c * kChunkWords + t;
                if (wd < words) pc += __popc(bm[wd]);
            }
            pc = wave_sum(pc);
            if (lane == 0 && first_chunk + c < nchunks) wcnt[(long long)blockIdx.x * nchunks + first_chunk + c] = pc;
            local += pc;
        }
        if (lane == 0 && local) atomicAdd(&s_row_total, local);
        __syncthreads();
    }
    if (threadIdx.x == 0) nnzc[row] = s_row_total;
}

// Split points of every B row at the numeric window boundaries:
// Bsplit[k * (nwin + 1) + w] = first position of row k with column >= w * W.
__global__ __launch_bounds__(256) void k_bsplit(int brows, int W, int nwin, const int *__restrict__ Brp,
                                                const int *__restrict__ Bcol, int *__restrict__ Bsplit)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = nwin + 1;
    if (t >= (long long)brows * per) return;
    const int k = (int)(t / per), w = (int)(t % per);
    const int b0 = Brp[k], b1 = Brp[k + 1];
    int pos;
    if (w == 0) pos = b0;
    else if (w == nwin) pos = b1;
    else pos = lower_bound_col(Bcol, b0, b1, w * W);
    Bsplit[t] = pos;
}

// Exclusive prefix of the chunk counts of every heavy row (row-relative output
// offsets of the chunks); one thread per heavy row.
__global__ __launch_bounds__(256) void k_chunk_prefix(int nheavy, int nchunks, const int *__restrict__ wcnt,
                                                      int *__restrict__ woff)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= nheavy) return;
    const long long base = (long long)h * nchunks;
    int run = 0;
    for (int c = 0; c < nchunks; ++c) {
        woff[base + c] = run;
        run += wcnt[base + c];
    }
}

// Numeric phase of heavy rows, windowed: block (h, w) accumulates the
// products of heavy row h whose columns fall in window w (UNITS chunks) into
// a dense LDS array plus an occupancy bitmap, then writes the window's
// entries in column order at their final offsets (bitmap rank).
template <typename V, int UNITS>
__global__ __launch_bounds__(kHeavyThreads) void k_num_heavy_dense(
    const int *__restrict__ Arp, const int *__restrict__ Acol, const V *__restrict__ Aval,
    const int *__restrict__ Bcol, const V *__restrict__ Bval, const int *__restrict__ Bsplit,
    const int *__restrict__ rows, int nwin, int nchunks, const int *__restrict__ wcnt,
    const int *__restrict__ woff, const long long *__restrict__ Crp, int *__restrict__ Ccol,
    V *__restrict__ Cval, int *err, int *nonempty)
{
    constexpr int W = UNITS * kChunkCols;
    constexpr int WORDS = W / 32;
    constexpr int NW = kHeavyThreads / kWave;
    constexpr int WPT = (WORDS + kHeavyThreads - 1) / kHeavyThreads;
    extern __shared__ unsigned char s_raw[];
    V *acc = (V *)s_raw;                                   // [W]
    unsigned *bm = (unsigned *)(acc + W);                  // [WORDS]
    int *s_incl = (int *)(bm + WORDS);                     // [NW][64]
    int *s_bs = s_incl + NW * kWave;                       // [NW][64]
    V *s_a = (V *)(s_bs + NW * kWave);                     // [NW][64]
    __shared__ long long s_tmp[kHeavyThreads / kWave + 1];
    const int h = blockIdx.x / nwin, w = blockIdx.x % nwin;
    const long long cb = (long long)h * nchunks;
    const int c0 = w * UNITS;
    int count = 0;
#pragma unroll
    for (int u = 0; u < UNITS; ++u)
        if (c0 + u < nchunks) count += wcnt[cb + c0 + u];
    if (count == 0) return;
    if (threadIdx.x == 0) atomicAdd(nonempty, 1);
    const int row = rows[h];
    const long long out0 = Crp[row] + woff[cb + c0];
    for (int t = threadIdx.x; t < W; t += kHeavyThreads) acc[t] = V(0);
    for (int t = threadIdx.x; t < WORDS; t += kHeavyThreads) bm[t] = 0u;
    __syncthreads();
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const int lo = w * W;
    const long long per = nwin + 1;
    wave_products<V, true>(
        Arp[row], Arp[row + 1], wave, NW, s_incl + wave * kWave, s_bs + wave * kWave, s_a + wave * kWave, Bcol, Bval,
        [&](int e, int &bs, int &bl, V &a) {
            const long long k = Acol[e];
            bs = Bsplit[k * per + w];
            bl = Bsplit[k * per + w + 1] - bs;
            a = Aval[e];
        },
        [&](int j, V p) {
            const int jl = j - lo;
            atomicAdd(&acc[jl], p);
            atomicOr(&bm[jl >> 5], 1u << (jl & 31));
        });
    __syncthreads();
    // rank of every set bit: thread t owns words [t*WPT, (t+1)*WPT)
    int pc = 0;
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
        const int wd = threadIdx.x * WPT + q;
        if (wd < WORDS) pc += __popc(bm[wd]);
    }
    long long tot;
    long long rank = block_excl_scan<long long, kHeavyThreads>((long long)pc, s_tmp, tot);
    if (threadIdx.x == 0 && tot != count) atomicOr(err, kErrCount);
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
        const int wd = threadIdx.x * WPT + q;
        if (wd >= WORDS) break;
        unsigned bits = bm[wd];
        while (bits) {
            const int b = __ffs(bits) - 1;
            bits &= bits - 1;
            const int jl = wd * 32 + b;
            if (rank < count) {
                Ccol[out0 + rank] = lo + jl;
                Cval[out0 + rank] = acc[jl];
            }
            ++rank;
        }
    }
    (void)lane;
}

// ---------------------------------------------- heavy rows: global hash path

__device__ __forceinline__ int gload(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename V>
__device__ __forceinline__ V gload_v(const V *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fills `n` ints with `v` (table initialisation).
__global__ __launch_bounds__(256) void k_fill_i32(long long n, int *__restrict__ p, int v)
{
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        p[t] = v;
}

template <typename V>
__global__ __launch_bounds__(256) void k_fill_zero(long long n, V *__restrict__ p)
{
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        p[t] = V(0);
}

// Symbolic phase of heavy rows in global mode: one block per row inserts the
// row's columns in its global key table (device-scope CAS) and counts them.
__global__ __launch_bounds__(kHeavyThreads) void k_sym_global(
    const int *__restrict__ Arp, const int *__restrict__ Acol, const int *__restrict__ Brp,
    const int *__restrict__ Bcol, const int *__restrict__ rows, const int *__restrict__ cap,
    const long long *__restrict__ goff, int *gkeys, int *__restrict__ nnzc, int *err)
{
    constexpr int NW = kHeavyThreads / kWave;
    __shared__ int s_incl[NW][kWave], s_bs[NW][kWave];
    __shared__ int s_cnt;
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const int row = rows[blockIdx.x];
    const int logT = gtable_log2(cap[row]);
    const unsigned mask = (1u << logT) - 1;
    int *keys = gkeys + goff[blockIdx.x];
    if (threadIdx.x == 0) s_cnt = 0;
    int mine = 0;
    wave_products<float, false>(
        Arp[row], Arp[row + 1], wave, NW, s_incl[wave], s_bs[wave], (float *)nullptr, Bcol, (const float *)nullptr,
        [&](int e, int &bs, int &bl, float &) {
            const int k = Acol[e];
            bs = Brp[k];
            bl = Brp[k + 1] - bs;
        },
        [&](int j) {
            unsigned hh = slot_of(j, logT);
            for (unsigned probe = 0; probe <= mask; ++probe) {
                int cur = gload(&keys[hh]);
                if (cur == j) return;
                if (cur == kEmpty) {
                    int old = atomicCAS(&keys[hh], kEmpty, j);
                    if (old == kEmpty) { ++mine; return; }
                    if (old == j) return;
                }
                hh = (hh + 1) & mask;
            }
            atomicOr(err, kErrProbe);
        });
    __syncthreads();
    mine = wave_sum(mine);
    if (lane == 0 && mine) atomicAdd(&s_cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) nnzc[row] = s_cnt;
}

// Numeric phase of heavy rows in global mode: one block per row clears its
// global tag/value table, merges the row's products into it with
// device-scope CAS and atomic add, then writes the entries in column order
// (rank from an LDS bitmap over column windows of kGlobalRankBits).
constexpr int kGlobalRankBits = 1 << 19;

template <typename V>
__global__ __launch_bounds__(kHeavyThreads) void k_num_global(
    const int *__restrict__ Arp, const int *__restrict__ Acol, const V *__restrict__ Aval,
    const int *__restrict__ Brp, const int *__restrict__ Bcol, const V *__restrict__ Bval,
    const int *__restrict__ rows, int ncols, const long long *__restrict__ goff, int *gkeys, V *gvals,
    const long long *__restrict__ Crp, int *__restrict__ Ccol, V *__restrict__ Cval, int *err)
{
    constexpr int NW = kHeavyThreads / kWave;
    constexpr int WORDS = kGlobalRankBits / 32;
    constexpr int WPT = WORDS / kHeavyThreads;
    extern __shared__ unsigned s_bm[];                     // [WORDS]
    __shared__ int s_incl[NW][kWave], s_bs[NW][kWave];
    __shared__ V s_a[NW][kWave];
    __shared__ long long s_tmp[kHeavyThreads / kWave + 1];
    __shared__ int s_base[kHeavyThreads];
    const int wave = threadIdx.x / kWave;
    const int row = rows[blockIdx.x];
    const long long rb = Crp[row];
    const int nc = (int)(Crp[row + 1] - rb);
    const int logT = gtable_log2(nc);
    const int T = 1 << logT;
    const unsigned mask = (unsigned)T - 1;
    int *keys = gkeys + goff[blockIdx.x];
    V *vals = gvals + goff[blockIdx.x];
    for (int t = threadIdx.x; t < T; t += kHeavyThreads) {
        keys[t] = kEmpty;
        vals[t] = V(0);
    }
    __threadfence();
    __syncthreads();
    wave_products<V, true>(
        Arp[row], Arp[row + 1], wave, NW, s_incl[wave], s_bs[wave], s_a[wave], Bcol, Bval,
        [&](int e, int &bs, int &bl, V &a) {
            const int k = Acol[e];
            bs = Brp[k];
            bl = Brp[k + 1] - bs;
            a = Aval[e];
        },
        [&](int j, V p) {
            unsigned hh = slot_of(j, logT);
            for (unsigned probe = 0; probe <= mask; ++probe) {
                int cur = gload(&keys[hh]);
                if (cur == kEmpty) {
                    int old = atomicCAS(&keys[hh], kEmpty, j);
                    cur = old == kEmpty ? j : old;
                }
                if (cur == j) {
                    atomicAdd(&vals[hh], p);
                    return;
                }
                hh = (hh + 1) & mask;
            }
            atomicOr(err, kErrProbe);
        });
    __threadfence();
    __syncthreads();
    long long done = 0;
    for (int lo = 0; lo < ncols; lo += kGlobalRankBits) {
        const int hi = lo + kGlobalRankBits < ncols ? lo + kGlobalRankBits : ncols;
        for (int t = threadIdx.x; t < WORDS; t += kHeavyThreads) s_bm[t] = 0u;
        __syncthreads();
        for (int t = threadIdx.x; t < T; t += kHeavyThreads) {
            const int j = gload(&keys[t]);
            if (j != kEmpty && j >= lo && j < hi) atomicOr(&s_bm[(j - lo) >> 5], 1u << ((j - lo) & 31));
        }
        __syncthreads();
        int pc = 0;
        for (int q = 0; q < WPT; ++q) pc += __popc(s_bm[threadIdx.x * WPT + q]);
        long long tot;
        const long long ex = block_excl_scan<long long, kHeavyThreads>((long long)pc, s_tmp, tot);
        s_base[threadIdx.x] = (int)ex;
        __syncthreads();
        for (int t = threadIdx.x; t < T; t += kHeavyThreads) {
            const int j = gload(&keys[t]);
            if (j == kEmpty || j < lo || j >= hi) continue;
            const int jl = j - lo, wd = jl >> 5, owner = wd / WPT;
            int rank = s_base[owner];
            for (int q = owner * WPT; q < wd; ++q) rank += __popc(s_bm[q]);
            rank += __popc(s_bm[wd] & ((1u << (jl & 31)) - 1u));
            const long long pos = done + rank;
            if (pos < nc) {
                Ccol[rb + pos] = j;
                Cval[rb + pos] = gload_v(&vals[t]);
            }
        }
        done += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && done != nc) atomicOr(err, kErrCount);
}

}  // namespace smash
