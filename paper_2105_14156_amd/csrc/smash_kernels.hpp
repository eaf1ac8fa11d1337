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
//   * a group of 64-lane wavefronts owns one output row (or one column
//     segment of a heavy row) and its LDS table; rows are binned by table
//     size so each bin launches a workgroup shape that fits its rows (the
//     paper's windows sized to the scratchpad);
//   * the products of a row are enumerated "flat": the group loads a chunk of
//     A's row, prefix-sums the lengths of the B rows it selects, and every
//     thread takes products q = t, t + G, ... of the concatenation, so a long
//     B row and many short ones keep every lane busy (the paper gives each
//     row two threads for the same reason, "SMASH Version 2: Tokenization");
//     several products per thread are loaded before any is merged, to keep
//     loads in flight;
//   * slots come from a multiplicative (Fibonacci) hash of the column, which
//     spreads clustered columns like the paper's low-order-bit hash of
//     version 2, with +1 linear probing;
//   * heavy rows (output bound above the LDS row limit) are cut into column
//     segments of at most kSegCap entries using per-8192-column counts from
//     the symbolic phase.  Sparse segments are hashed in LDS; chunks denser
//     than kSegCap are accumulated directly by column (the paper's per-row
//     dense/sparse decision of the Window Distribution Phase).  Optionally a
//     heavy row instead uses one hash table in global memory (version 3,
//     "Fragmenting Memory").
//   * output is written in column order: ranks from an occupancy bitmap of
//     the row's (or segment's) column range, built in the table's own LDS
//     once its entries are in registers, where that range is at most 64
//     times the table size, else a bitonic sort; dense chunks rank by
//     ballots over the accumulator; entries are staged in LDS so the global
//     stores are coalesced.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smash {

constexpr int kWave = 64;
constexpr int kEmpty = -1;              // empty-slot tag (Algorithm "SMASH SETUP": EMPTY = -1)
constexpr int kMinLogT = 6;             // smallest LDS row table: 64 slots
constexpr int kMaxLogT = 11;            // largest LDS row table: 2048 slots
constexpr int kLdsBins = kMaxLogT - kMinLogT + 1;
constexpr int kBinHeavy = kLdsBins;
constexpr int kBinEmpty = kLdsBins + 1;
constexpr int kNumBins = kLdsBins + 2;
constexpr int kChunkCols = 8192;        // column granularity of heavy-row counts
constexpr int kChunkWords = kChunkCols / 32;
constexpr int kSymWinChunks = 16;       // symbolic heavy window: 16 chunks, 16 KiB bitmap
constexpr int kSegCap = 1024;           // entries of one hashed segment (table of 2048 slots)
constexpr int kSegMerge = 600;          // chunks are merged into one segment up to this many entries
constexpr int kSegMaxSpan = 8;          // chunks spanned by one hashed segment
constexpr int kSegBins = 4;             // hashed segments with <=128, <=700, <=1024 entries; dense chunks
constexpr int kSegDense = 3;
constexpr int kBinBlockRows = 1024;     // rows per block of the binning kernels

enum : int {
    kErrProbe = 1,      // a hash table ran out of slots (inconsistent sizes)
    kErrCsrA = 2,       // A violates the CSR preconditions
    kErrCsrB = 4,       // B violates the CSR preconditions
    kErrCount = 8,      // numeric found a row count different from C_row_ptr
    kErrCapacity = 16,  // the workspace (or an output pool) is too small
};
// Conditions under which the rest of a pipeline must not run: its kernels
// test them on entry (the flags were set by earlier kernels of the same
// stream), so that no kernel indexes through an invalid matrix or beyond the
// workspace, and the host learns of it at its one synchronisation.
constexpr int kErrStop = kErrCsrA | kErrCsrB | kErrCapacity;

__device__ __forceinline__ bool stopped(const int *err)
{
    return err && (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrStop) != 0;
}

struct BinHdr {
    long long wsum[kNumBins]; // sum of the per-row weights (output entries) per bin
    int count[kNumBins];      // rows per bin
    int offset[kNumBins + 1]; // exclusive offsets of the bins in the row permutation
};

struct SegHdr {
    long long nnz[kSegBins];  // output entries per segment bin
    int count[kSegBins];
    int offset[kSegBins + 1];
};

struct DevHdr {
    unsigned long long products;       // sum over rows of products
    unsigned long long gneed[2];       // global-hash slots: [0] symbolic, [1] numeric
    long long nnz_c;
    long long stage_total;             // staging entries of the fused pass
    BinHdr sym, num, fz;
    SegHdr seg;
    int error;                         // flags of the symbolic pipeline
    int num_error;                     // flags of numeric calls, kept until read
    int fused_ok;                      // rows completed by the fused pass
    unsigned long long fused_entries;  // their entries
    // workspace query (smash_workspace_size): heavy rows, and the global
    // tables of the symbolic pass (total and largest, in slots)
    int q_heavy;
    unsigned long long q_gsum;
    unsigned long long q_gmax;
};

// A column segment of a heavy row: the row, its A entries, the chunk range,
// the number of output entries and their offset in C.
struct Seg {
    int row, e0, e1, c0, c1, count;
    long long out;
};

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Orders LDS accesses of one wavefront (lanes execute in lockstep; the fence
// keeps the compiler from moving LDS accesses across it).
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

// DPP controls of GFX9 (CDNA) used by the int scans below: shifts within
// rows of 16 lanes, broadcasts of lanes 15 and 31 to the following rows,
// and a whole-wave shift by one lane.
constexpr int kDppRowShr = 0x110;
constexpr int kDppBcast15 = 0x142;
constexpr int kDppBcast31 = 0x143;
constexpr int kDppWaveShr1 = 0x138;

// Inclusive scan over the 64 lanes of a wave with operator `op` and its
// identity `id`, in DPP moves (no LDS crossbar round trips): Hillis-Steele
// within each row of 16 lanes, then row 0's total into row 1 and row 2's
// into row 3, then rows 0-1's total into rows 2-3.
template <typename Op>
__device__ __forceinline__ int wave_scan_dpp(int v, int id, Op op)
{
    v = op(v, __builtin_amdgcn_update_dpp(id, v, kDppRowShr | 1, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(id, v, kDppRowShr | 2, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(id, v, kDppRowShr | 4, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(id, v, kDppRowShr | 8, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(id, v, kDppBcast15, 0xa, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(id, v, kDppBcast31, 0xc, 0xf, false));
    return v;
}

// The value of the lane below (lane 0 gets `id`).
__device__ __forceinline__ int wave_shift_up1(int v, int id)
{
    return __builtin_amdgcn_update_dpp(id, v, kDppWaveShr1, 0xf, 0xf, false);
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    if constexpr (sizeof(T) == 4) {
        return (T)wave_scan_dpp((int)v, 0, [](int a, int b) { return a + b; });
    } else {
        const int lane = lane_id();
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            T t = __shfl_up(v, d, kWave);
            if (lane >= d) v += t;
        }
        return v;
    }
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

// Output stores of C bypass cache retention: C is written once and never
// read back by the product, and keeping it out of L2 and the MALL leaves
// room for B and the split table, which every row re-reads.
template <typename T>
__device__ __forceinline__ void store_c(T *p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// Fibonacci hashing of a column index onto 2^logT slots.
__device__ __forceinline__ unsigned slot_of(int key, int logT)
{
    return ((unsigned)key * 2654435769u) >> (32 - logT);
}

// log2 of the global hash table size of a heavy row with at most n keys
// (load factor at most one half).
__host__ __device__ __forceinline__ int gtable_log2(long long n)
{
    long long x = 2 * (n > 1 ? n : 1);
    int l = 0;
    while ((1LL << l) < x) ++l;
    return l;
}

// Bin of a light row from its table bound (cap for symbolic, exact count for
// numeric): table of next_pow2(2 * bound) slots, at least 64.
__device__ __forceinline__ int lds_bin(long long bound)
{
    int lt = ceil_log2(2LL * bound);
    return (lt < kMinLogT ? kMinLogT : lt) - kMinLogT;
}

// Block-wide exclusive scan of one value per thread (all threads call it).
template <typename T, int THREADS>
__device__ __forceinline__ T block_excl_scan(T v, T *s_tmp /* THREADS/64 + 1 */, T &total)
{
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    T incl = wave_incl_scan(v);
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
// Shared LDS scratch of one group of G threads.
template <typename V, int G>
struct EnumScratch {
    int pincl[G];       // inclusive prefix of the piece counts of the long B ranges
    int sincl[G];       // inclusive prefix of the lengths of the short B ranges
    int bs[G];          // B range start of each A entry of the chunk
    int be[G];          // B range end of each A entry of the chunk
    V a[G];             // value of each A entry of the chunk
    int wsum[2 * (G / kWave)];
};

// Loads the U products of one thread (column, and value in double) with no
// branch between the loads, so all of them are in flight before the first is
// used.  A product with pos < 0 is absent; it loads entry 0 of B, which
// exists whenever the caller enumerates any product.
template <typename V, bool WITH_VAL, int U>
__device__ __forceinline__ void load_products(const int *__restrict__ Bcol, const V *__restrict__ Bval,
                                              const int (&pos)[U], int (&j)[U], double (&bv)[U])
{
    V raw[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int q = pos[u] >= 0 ? pos[u] : 0;
        j[u] = Bcol[q];
        if constexpr (WITH_VAL) raw[u] = Bval[q];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if constexpr (WITH_VAL) bv[u] = (double)raw[u];
        else bv[u] = 0.0;
    }
}

// Hands U loaded products of one thread to the sink: one call per product
// (sink(j, a * b), or sink(j) without values), or with ARRAY_SINK one call
// with all U (sink(j[U], p[U], ok[U]), or sink(j[U], ok[U])), so that the
// sink can overlap their LDS round trips.
template <bool WITH_VAL, int U, bool ARRAY_SINK, typename Sink>
__device__ __forceinline__ void emit_products(Sink &sink, const int (&pos)[U], const int (&j)[U],
                                              const double (&av)[U], const double (&bv)[U])
{
    if constexpr (ARRAY_SINK) {
        bool ok[U];
        double p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = pos[u] >= 0;
            p[u] = av[u] * bv[u];
        }
        if constexpr (WITH_VAL) sink(j, p, ok);
        else sink(j, ok);
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (pos[u] >= 0) {
                if constexpr (WITH_VAL) sink(j[u], av[u] * bv[u]);
                else sink(j[u]);
            }
        }
    }
}

// Calls sink(j, a * b) -- the product formed in double -- (or sink(j)
// without values) for every product of the A entries [e0, e1) of one row,
// each restricted to the B range returned by get(e, &bstart, &blen, &a).  The
// G threads of the group (thread index gt) take the row in chunks of G A
// entries.  B ranges of at least 64 entries are cut into pieces of 64
// products: each wave takes U consecutive pieces at a time, finds their A
// entry with one search that all its lanes share, and every lane loads one
// product per piece (coalesced, no per-lane search).  Shorter ranges, which
// carry few of the products, are enumerated flat: thread gt takes products
// q = gt, gt + G, ... and finds its A entry by binary search (consecutive
// lanes then read consecutive B entries where a range continues).  U products
// per thread are located and loaded before any is merged.
template <typename V, bool WITH_VAL, int G, int U, typename Get, typename Sink, bool ARRAY_SINK = false,
          bool PIPELINE = false>
__device__ __forceinline__ void group_products(int e0, int e1, int gt, EnumScratch<V, G> &S,
                                               const int *__restrict__ Bcol, const V *__restrict__ Bval,
                                               Get get, Sink sink)
{
    constexpr int WG = G / kWave;
    const int lane = lane_id(), wg = gt / kWave;
    for (int base = e0; base < e1; base += G) {
        const int e = base + gt;
        int bs = 0, bl = 0;
        V a = V(0);
        if (e < e1) get(e, bs, bl, a);
        const bool lng = bl >= kWave;
        int ip = wave_incl_scan(lng ? (bl + kWave - 1) / kWave : 0);
        int is = wave_incl_scan(lng ? 0 : bl);
        if constexpr (WG > 1) {
            if (lane == kWave - 1) {
                S.wsum[wg] = ip;
                S.wsum[WG + wg] = is;
            }
            group_sync<WG>();
            int ap = 0, as = 0;
            for (int w = 0; w < wg; ++w) {
                ap += S.wsum[w];
                as += S.wsum[WG + w];
            }
            ip += ap;
            is += as;
        }
        S.pincl[gt] = ip;
        S.sincl[gt] = is;
        S.bs[gt] = bs;
        S.be[gt] = bs + bl;
        if constexpr (WITH_VAL) S.a[gt] = a;
        group_sync<WG>();
        const int ptot = S.pincl[G - 1], stot = S.sincl[G - 1];
        // long ranges, piece by piece: wave wg takes U consecutive pieces per
        // round; with PIPELINE the pieces of the next round are located (LDS
        // searches) while the loads of this round are in flight.  A wave's
        // pieces only move forward, so it keeps a cursor `cur` (no piece of
        // it lies in an A entry before cur) and finds the A entry of piece
        // pc from one wave-wide read: lane l holds the boundary
        // pincl[cur + l - 1] (lane 0 the one before cur, never above pc),
        // and the first lane whose boundary exceeds pc names the entry.  One
        // read serves all U pieces of a round unless they run past it.
        int cur = 0;
        auto window = [&]() {
            const int t = cur + lane - 1;
            return t < 0 ? 0 : S.pincl[t < G ? t : G - 1];
        };
        auto locate_pieces = [&](int pc0, int (&pos)[U], double (&av)[U]) {
            int v = window();
            int last = cur;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int pc = pc0 + u;
                pos[u] = -1;
                av[u] = 0.0;
                if (pc < ptot) {                                   // wave-uniform
                    unsigned long long hit;
                    while (!(hit = __ballot(v > pc))) {
                        cur += kWave - 1;
                        v = window();
                    }
                    const int k = __ffsll((long long)hit) - 1;     // >= 1
                    const int src = cur + k - 1;
                    const int pex = __builtin_amdgcn_readlane(v, k - 1);
                    const int p = S.bs[src] + (pc - pex) * kWave + lane;
                    if (p < S.be[src]) {
                        pos[u] = p;
                        if constexpr (WITH_VAL) av[u] = (double)S.a[src];
                    }
                    last = src;
                }
            }
            cur = last;
        };
        {
            int pos[U];
            double av[U];
            int pc0 = wg * U;
            if constexpr (PIPELINE)
                if (pc0 < ptot) locate_pieces(pc0, pos, av);
            for (; pc0 < ptot; pc0 += WG * U) {
                int j[U];
                double bv[U];
                if constexpr (!PIPELINE) locate_pieces(pc0, pos, av);
                load_products<V, WITH_VAL, U>(Bcol, Bval, pos, j, bv);
                int posn[U];
                double avn[U];
                if constexpr (PIPELINE)
                    if (pc0 + WG * U < ptot) locate_pieces(pc0 + WG * U, posn, avn);
                emit_products<WITH_VAL, U, ARRAY_SINK>(sink, pos, j, av, bv);
                if constexpr (!PIPELINE) continue;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    pos[u] = posn[u];
                    av[u] = avn[u];
                }
            }
        }
        // short ranges, flat: thread gt takes products q = q0 + u * G + gt
        // and finds its A entry by binary search (consecutive lanes then read
        // consecutive B entries where a range continues); with PIPELINE the
        // next round is located while this round's loads are in flight
        auto locate_flat = [&](int q0, int (&pos)[U], double (&av)[U]) {
            // the U searches advance step by step together, so that their
            // LDS reads are in flight at once
            int src[U];
#pragma unroll
            for (int u = 0; u < U; ++u) src[u] = 0;
#pragma unroll
            for (int step = G / 2; step > 0; step >>= 1) {
                int t[U];
#pragma unroll
                for (int u = 0; u < U; ++u) t[u] = S.sincl[src[u] + step - 1];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (t[u] <= q0 + u * G + gt) src[u] += step;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + u * G + gt;
                pos[u] = -1;
                av[u] = 0.0;
                if (q < stot) {
                    const int excl = src[u] ? S.sincl[src[u] - 1] : 0;
                    pos[u] = S.bs[src[u]] + (q - excl);
                    if constexpr (WITH_VAL) av[u] = (double)S.a[src[u]];
                }
            }
        };
        {
            int pos[U];
            double av[U];
            if constexpr (PIPELINE)
                if (stot > 0) locate_flat(0, pos, av);
            for (int q0 = 0; q0 < stot; q0 += G * U) {
                int j[U];
                double bv[U];
                if constexpr (!PIPELINE) locate_flat(q0, pos, av);
                load_products<V, WITH_VAL, U>(Bcol, Bval, pos, j, bv);
                int posn[U];
                double avn[U];
                if constexpr (PIPELINE)
                    if (q0 + G * U < stot) locate_flat(q0 + G * U, posn, avn);
                emit_products<WITH_VAL, U, ARRAY_SINK>(sink, pos, j, av, bv);
                if constexpr (!PIPELINE) continue;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    pos[u] = posn[u];
                    av[u] = avn[u];
                }
            }
        }
        group_sync<WG>();
    }
}

// --------------------------------------------- product enumeration by runs
//
// run_products enumerates the same products as group_products with fewer
// instructions per product: locating a product's A entry (a search in LDS)
// is shared by 64 products of a wave (a full piece of a long range) or by
// the kRun consecutive products of one lane (a run of a short range), never
// done once per product.  Every B range is split into full pieces of 64
// products and a tail of fewer than 64; entries with full pieces form the
// long list, entries with a tail the short list (an entry can be in both),
// each compacted in LDS with the inclusive prefix of its piece (or run)
// counts.  Long phase: each wave locates 64 of its pieces at once, one per
// lane (a binary search over the long list, O(log n) reads per lane), keeps
// their starts in registers and then takes U pieces per step: the start of
// piece u is read across lanes (v_readlane) and lane l loads product
// start + l, coalesced.  Short phase: thread gt takes runs q = gt, gt + G,
// ... (RU per step), finds each run's entry by binary search over the short
// list and loads its kRun consecutive products.  Pieces are dealt to the
// waves U at a time in turn, so short rows still spread over the group.
constexpr int kRun = 4;

template <typename V, int GE, int G = GE>
struct RunScratch {
    int lincl[GE];  // long list: inclusive prefix of the full-piece counts
    int lbs[GE];    //   B range start
    V la[GE];       //   A value
    int sincl[GE];  // short list: inclusive prefix of the tail-run counts
    int sbs[GE];    //   start of the tail
    int sbe[GE];    //   end of the B range
    V sa[GE];       //   A value
    int wsum[3 * (G / kWave)];
};

// Number of entries of the strictly increasing incl[0, n) that are <= x,
// i.e. the first index whose prefix exceeds x (n is group-uniform).
__device__ __forceinline__ int prefix_rank(const int *incl, int n, int x)
{
    int lo = 0;
    for (int s = n > 0 ? 1 << (31 - __clz(n)) : 0; s > 0; s >>= 1)
        if (lo + s <= n && incl[lo + s - 1] <= x) lo += s;
    return lo;
}

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// GE (a multiple of 64, at most G) is the number of A entries taken per step;
// a group with more threads than entries per step keeps the LDS lists small
// while all G threads share the products.
template <typename V, bool WITH_VAL, int GE, int G, int U, int RU, int RUN, typename Get, typename Sink,
          bool ARRAY_SINK = false>
__device__ __forceinline__ void run_products(int e0, int e1, int gt, RunScratch<V, GE, G> &S,
                                             const int *__restrict__ Bcol, const V *__restrict__ Bval, Get get,
                                             Sink sink)
{
    constexpr int WG = G / kWave;
    static_assert(kWave % U == 0, "U must divide the wave");
    static_assert(GE % kWave == 0 && GE <= G, "entry step");
    const int lane = lane_id(), wg = gt / kWave;
    for (int base = e0; base < e1; base += GE) {
        const int e = base + gt;
        int bs = 0, bl = 0;
        V a = V(0);
        if (gt < GE && e < e1) get(e, bs, bl, a);
        const int np = bl >> 6;                          // full pieces
        const int tail = bl & (kWave - 1);
        const int nr = (tail + RUN - 1) / RUN;           // runs of the tail
        const int isl = np > 0, iss = tail > 0;
        int ip = wave_incl_scan(np);
        int ic = wave_incl_scan(isl | (iss << 16));
        int ir = wave_incl_scan(nr);
        int P, RT, NC;
        if constexpr (WG > 1) {
            if (lane == kWave - 1) {
                S.wsum[wg] = ip;
                S.wsum[WG + wg] = ic;
                S.wsum[2 * WG + wg] = ir;
            }
            group_sync<WG>();
            int ap = 0, ac = 0, ar = 0;
            P = 0, NC = 0, RT = 0;
            for (int w = 0; w < WG; ++w) {
                const int tp = S.wsum[w], tc = S.wsum[WG + w], tr = S.wsum[2 * WG + w];
                if (w < wg) { ap += tp; ac += tc; ar += tr; }
                P += tp;
                NC += tc;
                RT += tr;
            }
            ip += ap;
            ic += ac;
            ir += ar;
        } else {
            P = __builtin_amdgcn_readlane(ip, kWave - 1);
            NC = __builtin_amdgcn_readlane(ic, kWave - 1);
            RT = __builtin_amdgcn_readlane(ir, kWave - 1);
        }
        const int NL = NC & 0xffff, NS = NC >> 16;
        if (isl) {
            const int li = (ic & 0xffff) - 1;
            S.lincl[li] = ip;
            S.lbs[li] = bs;
            if constexpr (WITH_VAL) S.la[li] = a;
        }
        if (iss) {
            const int si = (ic >> 16) - 1;
            S.sincl[si] = ir;
            S.sbs[si] = bs + (np << 6);
            S.sbe[si] = bs + bl;
            if constexpr (WITH_VAL) S.sa[si] = a;
        }
        group_sync<WG>();
        // long phase: wave wg owns pieces (k * WG + wg) * U + u, k = 0, 1, ...
        for (int k0 = 0; (k0 * WG + wg) * U < P; k0 += kWave / U) {
            const int pc = ((k0 + lane / U) * WG + wg) * U + lane % U;
            int st = -1;
            double al = 0.0;
            if (pc < P) {
                const int li = prefix_rank(S.lincl, NL, pc);
                const int ex = li ? S.lincl[li - 1] : 0;
                st = S.lbs[li] + ((pc - ex) << 6);
                if constexpr (WITH_VAL) al = (double)S.la[li];
            }
            for (int g = 0; g < kWave / U && ((k0 + g) * WG + wg) * U < P; ++g) {
                int pos[U], j[U];
                double av[U], bv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int s = __builtin_amdgcn_readlane(st, g * U + u);
                    pos[u] = s >= 0 ? s + lane : -1;
                    if constexpr (WITH_VAL) av[u] = readlane_d(al, g * U + u);
                    else av[u] = 0.0;
                }
                load_products<V, WITH_VAL, U>(Bcol, Bval, pos, j, bv);
                emit_products<WITH_VAL, U, ARRAY_SINK>(sink, pos, j, av, bv);
            }
        }
        // short phase: runs of kRun consecutive products of the tails
        for (int q0 = 0; q0 < RT; q0 += G * RU) {
            int src[RU];
#pragma unroll
            for (int r = 0; r < RU; ++r) src[r] = 0;
            // the RU searches advance together (their LDS reads overlap)
            for (int s = NS > 0 ? 1 << (31 - __clz(NS)) : 0; s > 0; s >>= 1) {
                int t[RU];
#pragma unroll
                for (int r = 0; r < RU; ++r) t[r] = src[r] + s <= NS ? S.sincl[src[r] + s - 1] : 0x7fffffff;
#pragma unroll
                for (int r = 0; r < RU; ++r)
                    if (t[r] <= q0 + r * G + gt) src[r] += s;
            }
            constexpr int N = RU * RUN;
            int pos[N], j[N];
            double av[N], bv[N];
#pragma unroll
            for (int r = 0; r < RU; ++r) {
                const int q = q0 + r * G + gt;
                int st = 0, en = 0;
                double ar = 0.0;
                if (q < RT) {
                    const int ex = src[r] ? S.sincl[src[r] - 1] : 0;
                    st = S.sbs[src[r]] + (q - ex) * RUN;
                    en = S.sbe[src[r]];
                    if constexpr (WITH_VAL) ar = (double)S.sa[src[r]];
                }
#pragma unroll
                for (int i = 0; i < RUN; ++i) {
                    pos[r * RUN + i] = st + i < en ? st + i : -1;
                    av[r * RUN + i] = ar;
                }
            }
            load_products<V, WITH_VAL, N>(Bcol, Bval, pos, j, bv);
            emit_products<WITH_VAL, N, ARRAY_SINK>(sink, pos, j, av, bv);
        }
        group_sync<WG>();
    }
}

// ------------------------------------------------------------ LDS hashing

// Claims the slot of `key` in an LDS key table, probing from slot h; returns
// 1 if the key was new.
__device__ __forceinline__ int lds_insert_key_at(int *keys, int logT, int key, unsigned h, int *err)
{
    const unsigned mask = (1u << logT) - 1;
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

__device__ __forceinline__ int lds_insert_key(int *keys, int logT, int key, int *err)
{
    return lds_insert_key_at(keys, logT, key, slot_of(key, logT), err);
}

// Claims or finds the slot of `key`, probing from slot h, and adds `p` to its
// value (values are accumulated in double: the LDS FP64 atomic add is the
// fast one on gfx950).
__device__ __forceinline__ void lds_insert_add_at(int *keys, double *vals, int logT, int key, double p, unsigned h,
                                                  int *err)
{
    const unsigned mask = (1u << logT) - 1;
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

__device__ __forceinline__ void lds_insert_add(int *keys, double *vals, int logT, int key, double p, int *err)
{
    lds_insert_add_at(keys, vals, logT, key, p, slot_of(key, logT), err);
}

// U products of one thread at once, each starting with a compare-and-swap
// of its home slot (empty -> column), all U issued before any result is
// used: the CAS returns the slot's previous key, so one LDS round trip tells
// whether the column was claimed (empty), is already there (its key), or
// met another column (probing continues one product at a time from the next
// slot).  Two products of the same column in one thread are safe: the
// second CAS returns the first one's key.
template <int U>
__device__ __forceinline__ void lds_insert_add_u(int *keys, double *vals, int logT, const int (&j)[U],
                                                 const double (&p)[U], const bool (&ok)[U], int *err)
{
    const unsigned mask = (1u << logT) - 1;
    unsigned h[U];
    int old[U];
#pragma unroll
    for (int u = 0; u < U; ++u) h[u] = slot_of(j[u], logT);
#pragma unroll
    for (int u = 0; u < U; ++u) old[u] = ok[u] ? atomicCAS(&keys[h[u]], kEmpty, j[u]) : j[u];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (!ok[u]) continue;
        if (old[u] == kEmpty || old[u] == j[u]) atomicAdd(&vals[h[u]], p[u]);
        else lds_insert_add_at(keys, vals, logT, j[u], p[u], (h[u] + 1) & mask, err);
    }
}

// Key-only variant: returns how many of the U columns were new.
template <int U>
__device__ __forceinline__ int lds_insert_key_u(int *keys, int logT, const int (&j)[U], const bool (&ok)[U], int *err)
{
    const unsigned mask = (1u << logT) - 1;
    unsigned h[U];
    int old[U];
    int added = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) h[u] = slot_of(j[u], logT);
#pragma unroll
    for (int u = 0; u < U; ++u) old[u] = ok[u] ? atomicCAS(&keys[h[u]], kEmpty, j[u]) : j[u];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (!ok[u]) continue;
        if (old[u] == kEmpty) ++added;
        else if (old[u] != j[u]) added += lds_insert_key_at(keys, logT, j[u], (h[u] + 1) & mask, err);
    }
    return added;
}

// Order-preserving variant (the paper's first version, High-Bit Hashing):
// the home slot of column j is j >> shift, so slots rise with the column;
// CAS-first like lds_insert_add_u, then +1 linear probing (modulo T).  The
// longest probe distance of the row is kept in *maxd: the table is then
// sorted except within that distance (see order_row_entries_ord).
template <int U>
__device__ __forceinline__ void lds_insert_add_ord_u(int *keys, double *vals, int logT, int shift, const int (&j)[U],
                                                     const double (&p)[U], const bool (&ok)[U], int *maxd, int *err)
{
    const unsigned mask = (1u << logT) - 1;
    unsigned h[U];
    int old[U];
#pragma unroll
    for (int u = 0; u < U; ++u) h[u] = ((unsigned)j[u] >> shift) & mask;
#pragma unroll
    for (int u = 0; u < U; ++u) old[u] = ok[u] ? atomicCAS(&keys[h[u]], kEmpty, j[u]) : j[u];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (!ok[u]) continue;
        if (old[u] == kEmpty || old[u] == j[u]) {
            atomicAdd(&vals[h[u]], p[u]);
            continue;
        }
        unsigned hh = h[u];
        bool placed = false;
        for (unsigned d = 1; d <= mask; ++d) {
            hh = (hh + 1) & mask;
            int cur = __hip_atomic_load(&keys[hh], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (cur == kEmpty) {
                const int o = atomicCAS(&keys[hh], kEmpty, j[u]);
                cur = o == kEmpty ? j[u] : o;
            }
            if (cur == j[u]) {
                atomicAdd(&vals[hh], p[u]);
                if ((int)d > __hip_atomic_load(maxd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                    atomicMax(maxd, (int)d);
                placed = true;
                break;
            }
        }
        if (!placed) atomicOr(err, kErrProbe);
    }
}

// --------------------------------------------------------------- validation

// CSR preconditions of one matrix in two passes (a violation sets `flag` in
// *err).  Rows, one thread per row: row_ptr starts at 0, ends at nnz and
// never decreases; the first entry of every non-empty row is marked in a
// bitmap over the entries (cleared beforehand).  Entries, one thread per
// entry (coalesced): the column is in range and above the previous entry's
// unless the entry starts a row.  Without a bitmap (starts = NULL) only what
// memory safety needs is checked: row pointers and column ranges.
__global__ __launch_bounds__(256) void k_validate_rows(int rows, long long nnz, const int *__restrict__ rp,
                                                       unsigned *__restrict__ starts, int flag, int *err)
{
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (r == 0 && (rp[0] != 0 || (long long)rp[rows] != nnz)) bad = true;
    if (r < rows) {
        const int a = rp[r], b = rp[r + 1];
        if (b < a || a < 0 || (long long)b > nnz) bad = true;
        else if (a < b && starts) atomicOr(&starts[a >> 5], 1u << (a & 31));
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(err, flag);
}

__global__ __launch_bounds__(256) void k_validate_cols(int cols, long long nnz, const int *__restrict__ ci,
                                                       const unsigned *__restrict__ starts, int flag, int *err)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (p < nnz) {
        const int c = ci[p];
        if (c < 0 || c >= cols) bad = true;
        else if (starts && p > 0 && c <= ci[p - 1] && !((starts[p >> 5] >> (p & 31)) & 1u)) bad = true;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(err, flag);
}

// --------------------------------------------------------- analysis & bins

// Feature t (0..5) of the learned predictor for a row with na A entries:
// log2(1 + x) of na, the products ub, max_k nnz(B_k), min_k nnz(B_k),
// min(ub, cols) and sum_k nnz(B_k)^2 / ub, in double, rounded to float; 0 for
// a row without entries.  The selection is branch-free so that six lanes
// evaluate their features together.
__device__ __forceinline__ float row_feature(int t, int na, long long ub, double sq, int mx, int mn, int ncols)
{
    if (na == 0) return 0.f;
    const double cap = ub < ncols ? (double)ub : (double)ncols;
    const double x = t == 0 ? (double)na
                   : t == 1 ? (double)ub
                   : t == 2 ? (double)mx
                   : t == 3 ? (double)mn
                   : t == 4 ? cap
                            : (ub > 0 ? sq / (double)ub : 0.0);
    return (float)log2(1.0 + x);
}

// Row analysis (step a1): products ub_i = sum_k nnz(B_k) over row i of A, the
// output bound cap_i = min(ub_i, cols) and the row's symbolic bin.  A wave
// takes eight rows: rows of at most 64 entries are summed by their own group
// of eight lanes (most rows of A have a few dozen entries, so a whole wave
// per row would leave most lanes idle), longer rows one after another by the
// whole wave, four entries per lane in flight, so that a hub row does not
// leave one group with a long serial chain.  With feats non-NULL it also
// writes the learned predictor's six features and max_k nnz(B_k) (maxb_out)
// of the rows whose bound exceeds the LDS row limit, the only rows the
// predictor is asked about.
constexpr int kRowLanes = 8;
constexpr int kShortRow = 64;

// Partial sums of one lane over entries e0 + first, e0 + first + step, ...
struct RowPart {
    long long ub = 0;
    double sq = 0.0;
    int mx = 0, mn = 0x7fffffff;
};

template <bool FEATS>
__device__ __forceinline__ void row_part(const int *__restrict__ Acol, const int *__restrict__ Brp, int e, int e1,
                                         int step, RowPart &r)
{
    for (; e + 3 * step < e1; e += 4 * step) {
        int k[4], len[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) k[u] = Acol[e + u * step];
#pragma unroll
        for (int u = 0; u < 4; ++u) len[u] = Brp[k[u] + 1] - Brp[k[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            r.ub += len[u];
            if constexpr (FEATS) {
                r.sq += (double)len[u] * (double)len[u];
                r.mx = len[u] > r.mx ? len[u] : r.mx;
                r.mn = len[u] < r.mn ? len[u] : r.mn;
            }
        }
    }
    for (; e < e1; e += step) {
        const int len = Brp[Acol[e] + 1] - Brp[Acol[e]];
        r.ub += len;
        if constexpr (FEATS) {
            r.sq += (double)len * (double)len;
            r.mx = len > r.mx ? len : r.mx;
            r.mn = len < r.mn ? len : r.mn;
        }
    }
}

// Reduction of RowPart over lanes that differ in the bits of `width - 1`.
template <bool FEATS>
__device__ __forceinline__ void row_reduce(RowPart &r, int width)
{
    for (int d = width / 2; d > 0; d >>= 1) {
        r.ub += __shfl_xor(r.ub, d, kWave);
        if constexpr (FEATS) {
            r.sq += __shfl_xor(r.sq, d, kWave);
            const int a = __shfl_xor(r.mx, d, kWave), b = __shfl_xor(r.mn, d, kWave);
            r.mx = a > r.mx ? a : r.mx;
            r.mn = b < r.mn ? b : r.mn;
        }
    }
}

// Sums of the wave's eight rows [row0, row0 + 8) into the lanes of each
// row's group (every lane of the wave calls it).
template <bool FEATS>
__device__ __forceinline__ RowPart wave_rows(int m, int row0, const int *__restrict__ Arp,
                                             const int *__restrict__ Acol, const int *__restrict__ Brp, int &e0,
                                             int &e1)
{
    const int lane = lane_id(), sl = lane & (kRowLanes - 1), row = row0 + lane / kRowLanes;
    e0 = row < m ? Arp[row] : 0;
    e1 = row < m ? Arp[row + 1] : 0;
    const bool lng = e1 - e0 > kShortRow;
    RowPart r;
    if (!lng) row_part<FEATS>(Acol, Brp, e0 + sl, e1, kRowLanes, r);
    row_reduce<FEATS>(r, kRowLanes);
    unsigned long long todo = __ballot(lng && sl == 0);
    while (todo) {
        const int src = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        RowPart w;
        row_part<FEATS>(Acol, Brp, __builtin_amdgcn_readlane(e0, src) + lane, __builtin_amdgcn_readlane(e1, src),
                        kWave, w);
        row_reduce<FEATS>(w, kWave);
        if (lane / kRowLanes == src / kRowLanes) r = w;
    }
    return r;
}

__global__ __launch_bounds__(256) void k_analyze(int m, int ncols, int lds_row_max,
                                                 const int *__restrict__ Arp, const int *__restrict__ Acol,
                                                 const int *__restrict__ Brp, long long *__restrict__ ub_out,
                                                 int *__restrict__ cap_out, int *__restrict__ nnzc,
                                                 unsigned char *__restrict__ bin_out, float *__restrict__ feats,
                                                 int *__restrict__ maxb_out, const int *err)
{
    const int row0 = (blockIdx.x * 256 + (int)threadIdx.x) / kWave * kRowLanes;
    if (row0 >= m || stopped(err)) return;               // whole waves
    const int sl = lane_id() & (kRowLanes - 1), row = row0 + lane_id() / kRowLanes;
    int e0, e1;
    RowPart r = feats ? wave_rows<true>(m, row0, Arp, Acol, Brp, e0, e1)
                      : wave_rows<false>(m, row0, Arp, Acol, Brp, e0, e1);
    if (row >= m) return;
    const long long ub = r.ub;
    if (feats && (ub < ncols ? ub : ncols) > lds_row_max) {
        // the predictor's six features (the same arithmetic as k_features):
        // lanes 0..5 of the row's group write one each
        if (sl < 6) feats[(long long)row * 6 + sl] = row_feature(sl, e1 - e0, ub, r.sq, r.mx, r.mn, ncols);
        if (sl == 0) maxb_out[row] = e1 > e0 ? r.mx : 0;
    }
    if (sl == 0) {
        const int cap = (int)(ub < ncols ? ub : ncols);
        int b;
        if (ub == 0) b = kBinEmpty;
        else if (cap > lds_row_max) b = kBinHeavy;
        else b = lds_bin(cap);
        ub_out[row] = ub;
        cap_out[row] = cap;
        nnzc[row] = 0;
        bin_out[row] = (unsigned char)b;
    }
}

// Workspace query (smash_workspace_size): the number of heavy rows and the
// slots their global tables would take (total and largest), from the same
// bounds as k_analyze (eight rows per wave, grid-stride over whole waves);
// the counts of a block's rows are summed in LDS and added with one atomic
// per block and counter.
__global__ __launch_bounds__(256) void k_ws_query(int m, int ncols, int lds_row_max, const int *__restrict__ Arp,
                                                  const int *__restrict__ Acol, const int *__restrict__ Brp,
                                                  DevHdr *h)
{
    constexpr int RPB = 256 / kWave * kRowLanes;        // rows per block and step
    __shared__ unsigned long long s_sum[256 / kWave], s_max[256 / kWave];
    __shared__ int s_cnt[256 / kWave];
    const int lane = lane_id(), w = threadIdx.x / kWave, sl = lane & (kRowLanes - 1);
    int cnt = 0;
    unsigned long long gsum = 0, gmax = 0;
    if (!stopped(&h->error)) {
        for (int r0 = blockIdx.x * RPB + w * kRowLanes; r0 < m; r0 += gridDim.x * RPB) {
            int e0, e1;
            const RowPart r = wave_rows<false>(m, r0, Arp, Acol, Brp, e0, e1);
            const int row = r0 + lane / kRowLanes;
            const long long cap = r.ub < ncols ? r.ub : ncols;
            if (row < m && sl == 0 && cap > lds_row_max) {
                const unsigned long long t = 1ull << gtable_log2(cap);
                ++cnt;
                gsum += t;
                gmax = t > gmax ? t : gmax;
            }
        }
    }
    // wave totals, then the block's
    for (int d = kWave / 2; d > 0; d >>= 1) {
        cnt += __shfl_xor(cnt, d, kWave);
        gsum += __shfl_xor(gsum, d, kWave);
        const unsigned long long o = __shfl_xor(gmax, d, kWave);
        gmax = o > gmax ? o : gmax;
    }
    if (lane == 0) {
        s_cnt[w] = cnt;
        s_sum[w] = gsum;
        s_max[w] = gmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < 256 / kWave; ++v) {
            cnt += s_cnt[v];
            gsum += s_sum[v];
            gmax = s_max[v] > gmax ? s_max[v] : gmax;
        }
        if (cnt) {
            atomicAdd(&h->q_heavy, cnt);
            atomicAdd(&h->q_gsum, gsum);
            atomicMax(&h->q_gmax, gmax);
        }
    }
}

// Numeric bin of every row from its exact count (heavy rows stay heavy).
__global__ __launch_bounds__(256) void k_num_bins(int m, const int *__restrict__ nnzc,
                                                  const unsigned char *__restrict__ sym_bin_of,
                                                  unsigned char *__restrict__ bin_out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int b = sym_bin_of[i];
    const int nc = nnzc[i];
    // rows outside the plan (no products, or completed by the fused pass) stay out
    bin_out[i] = (unsigned char)(b == kBinHeavy ? kBinHeavy : (b == kBinEmpty || nc == 0 ? kBinEmpty : lds_bin(nc)));
}

// Per-block bin histograms (kBinBlockRows rows per block, no global atomics):
// bcount[blk * kNumBins + b], the block's per-bin sum of the row weights wt
// (bw, when wt is given) and the block's sum of products (bprod, when ub is
// given).
__global__ __launch_bounds__(256) void k_bin_count(int m, const unsigned char *__restrict__ bin_of,
                                                   const long long *__restrict__ ub, const int *__restrict__ wt,
                                                   int *__restrict__ bcount, unsigned long long *__restrict__ bprod,
                                                   long long *__restrict__ bw, const int *err)
{
    if (stopped(err)) return;
    __shared__ int s_hist[kNumBins];
    __shared__ unsigned long long s_w[kNumBins];
    __shared__ unsigned long long s_prod;
    if (threadIdx.x < kNumBins) {
        s_hist[threadIdx.x] = 0;
        s_w[threadIdx.x] = 0;
    }
    if (threadIdx.x == 0) s_prod = 0;
    __syncthreads();
    unsigned long long prod = 0;
    for (int r = threadIdx.x; r < kBinBlockRows; r += 256) {
        const long long i = (long long)blockIdx.x * kBinBlockRows + r;
        if (i < m) {
            const int b = bin_of[i];
            atomicAdd(&s_hist[b], 1);
            if (wt) atomicAdd(&s_w[b], (unsigned long long)wt[i]);
            if (ub) prod += (unsigned long long)ub[i];
        }
    }
    prod = wave_sum(prod);
    if (lane_id() == 0 && prod) atomicAdd(&s_prod, prod);
    __syncthreads();
    if (threadIdx.x < kNumBins) {
        bcount[blockIdx.x * kNumBins + threadIdx.x] = s_hist[threadIdx.x];
        if (bw) bw[blockIdx.x * kNumBins + threadIdx.x] = (long long)s_w[threadIdx.x];
    }
    if (threadIdx.x == 0 && bprod) bprod[blockIdx.x] = s_prod;
}

// Bin totals and offsets, and every block's base inside each bin (one block).
__global__ __launch_bounds__(256) void k_bin_scan(int nblk, int *__restrict__ bcount,
                                                  const unsigned long long *__restrict__ bprod,
                                                  const long long *__restrict__ bw, BinHdr *h,
                                                  unsigned long long *products, int *err, long long heavy_cap)
{
    // err: with heavy_cap >= 0, more heavy rows than the workspace holds
    // raise kErrCapacity (every later kernel of the pipeline then stops)
    if (stopped(err)) return;
    __shared__ int s_tot[kNumBins];
    __shared__ long long s_wt[kNumBins];
    // one wave per bin scans the block counts in place (exclusive)
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    for (int b = wave; b < kNumBins; b += 256 / kWave) {
        int run = 0;
        for (int c0 = 0; c0 < nblk; c0 += kWave) {
            const int c = c0 + lane;
            const int v = c < nblk ? bcount[c * kNumBins + b] : 0;
            const int incl = wave_incl_scan(v);
            if (c < nblk) bcount[c * kNumBins + b] = run + incl - v;
            run += __shfl(incl, kWave - 1, kWave);
        }
        long long ws = 0;
        if (bw)
            for (int c = lane; c < nblk; c += kWave) ws += bw[c * kNumBins + b];
        ws = wave_sum(ws);
        if (lane == 0) {
            s_tot[b] = run;
            s_wt[b] = ws;
        }
    }
    unsigned long long p = 0;
    if (bprod)
        for (int c = threadIdx.x; c < nblk; c += 256) p += bprod[c];
    p = wave_sum(p);
    __shared__ unsigned long long s_p[4];
    if (lane == 0) s_p[wave] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int b = 0; b < kNumBins; ++b) {
            h->count[b] = s_tot[b];
            h->wsum[b] = s_wt[b];
            h->offset[b] = run;
            run += s_tot[b];
        }
        h->offset[kNumBins] = run;
        if (bprod && products) *products = s_p[0] + s_p[1] + s_p[2] + s_p[3];
        if (err && heavy_cap >= 0 && s_tot[kBinHeavy] > heavy_cap) atomicOr(err, kErrCapacity);
    }
}

// Groups row ids by bin (empty rows are left out): perm[offset[b] + block base
// + rank in block].  For the heavy bin, also records the row's global-hash
// table size (gsz, by heavy index) when gsize_of is given.
__global__ __launch_bounds__(256) void k_scatter(int m, const unsigned char *__restrict__ bin_of,
                                                 const int *__restrict__ bbase, const BinHdr *h,
                                                 int *__restrict__ perm, const int *__restrict__ gsize_of,
                                                 long long *__restrict__ gsz, const int *err)
{
    if (stopped(err)) return;
    __shared__ int s_cnt[kNumBins];
    if (threadIdx.x < kNumBins) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int r = threadIdx.x; r < kBinBlockRows; r += 256) {
        const long long i = (long long)blockIdx.x * kBinBlockRows + r;
        if (i >= m) break;
        const int b = bin_of[i];
        const int local = atomicAdd(&s_cnt[b], 1);
        if (b == kBinEmpty) continue;
        const int pos = h->offset[b] + bbase[blockIdx.x * kNumBins + b] + local;
        perm[pos] = (int)i;
        if (b == kBinHeavy && gsize_of) gsz[pos - h->offset[kBinHeavy]] = 1LL << gtable_log2(gsize_of[i]);
    }
}

// ------------------------------------------------------- symbolic, LDS hash

// Symbolic count of one light row by a group of WPR waves (gt: thread index
// in the group; every thread of the group calls it): the distinct columns of
// the row's A entries [e0, e1) times B, counted in an LDS key table of
// 2^LOGT slots (step a3), are stored to *out by the group's first thread.
template <int LOGT, int WPR>
__device__ __forceinline__ void sym_row(int e0, int e1, const int *__restrict__ Acol, const int *__restrict__ Brp,
                                        const int *__restrict__ Bcol, bool active, int gt, int *keys,
                                        EnumScratch<float, WPR * kWave> &en, int *s_cnt, int *out, int *err)
{
    constexpr int T = 1 << LOGT;
    constexpr int G = WPR * kWave;
    for (int t = gt; t < T; t += G) keys[t] = kEmpty;
    if (gt == 0) *s_cnt = 0;
    group_sync<WPR>();
    int mine = 0;
    if (active) {
        auto get = [&](int e, int &bs, int &bl, float &) {
            const int k = Acol[e];
            bs = Brp[k];
            bl = Brp[k + 1] - bs;
        };
        auto sink = [&](const int (&j)[2], const bool (&ok)[2]) { mine += lds_insert_key_u<2>(keys, LOGT, j, ok, err); };
        group_products<float, false, G, 2, decltype(get), decltype(sink), true>(e0, e1, gt, en, Bcol,
                                                                                (const float *)nullptr, get, sink);
    }
    mine = wave_sum(mine);
    if (lane_id() == 0 && mine) atomicAdd(s_cnt, mine);
    group_sync<WPR>();
    if (active && gt == 0) *out = *s_cnt;
}

// Light rows of bin `bin`: one row per group of WPR waves (RPW groups per
// block; RPW > 1 only with WPR = 1).  The grid is persistent: the bin's rows
// and their number come from the device (perm + h->offset[bin],
// h->count[bin]) and the groups stride over them, so the launch needs no
// host-side count.  With RPW > 1 each group is one wave and loops on its
// own; with WPR > 1 the block is one group and loops as a whole.
template <int LOGT, int WPR, int RPW>
__global__ __launch_bounds__(kWave *WPR *RPW) void k_sym_rows(const int *__restrict__ Arp, const int *__restrict__ Acol,
                                                              const int *__restrict__ Brp, const int *__restrict__ Bcol,
                                                              const int *__restrict__ perm, const BinHdr *h, int bin,
                                                              int *__restrict__ nnzc, int *err)
{
    static_assert(RPW == 1 || WPR == 1, "multi-row blocks use one wave per row");
    constexpr int G = WPR * kWave;
    if (stopped(err)) return;
    __shared__ int s_keys[RPW][1 << LOGT];
    __shared__ EnumScratch<float, G> s_en[RPW];
    __shared__ int s_cnt[RPW];
    const int g = threadIdx.x / kWave / WPR;
    const int gt = threadIdx.x - g * G;
    const int nrows = h->count[bin];
    const int *rows = perm + h->offset[bin];
    for (int r0 = blockIdx.x * RPW; r0 < nrows; r0 += gridDim.x * RPW) {
        const int r = r0 + g;
        const bool active = r < nrows;
        const int row = active ? rows[r] : 0;
        const int e0 = active ? Arp[row] : 0, e1 = active ? Arp[row + 1] : 0;
        sym_row<LOGT, WPR>(e0, e1, Acol, Brp, Bcol, active, gt, s_keys[g], s_en[g], &s_cnt[g], &nnzc[row], err);
        group_sync<WPR>();
    }
}

// -------------------------------------------------------- numeric, LDS hash

// Key-value bitonic sort of n2 (a power of two) LDS entries by a group of G
// threads whose index in the group is gt.
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

// Puts the entries of a row's table in column order at the front of the
// table (keys[0 .. total), vals[0 .. total)).  kr/vr hold each thread's SPT
// slots of the table (kEmpty where free), cnt/incl/wbase their count, its
// inclusive wave prefix and the wave's offset in the group; every thread of
// the group calls it.  The columns lie in [lo, lo + ncols).  With ncols at
// most 64 T the order comes from ranks in an occupancy bitmap over that
// range built in the table's own LDS; otherwise the entries are compacted
// and sorted (bitonic), or, for one wave and at most 64 entries, ranked by
// counting the smaller columns across the wave's lanes.  Only that second
// form reads total, cnt, incl and wbase.  Returns the number of entries:
// the bitmap's count, or total.
template <int T, int WPR, int SPT>
__device__ __forceinline__ int order_row_entries(const int (&kr)[SPT], const double (&vr)[SPT], int *keys,
                                                 double *vals, int *s_scan, int total, int wbase, int incl, int cnt,
                                                 int ncols, int gt, int lo = 0)
{
    constexpr int G = WPR * kWave;
    const int lane = lane_id(), wg = gt / kWave;
    group_sync<WPR>();
    if (ncols <= 64 * T) {
        // bitmap over B's columns in the value area (2T words), the prefix
        // of its popcounts per word (16-bit) in the key area; then every
        // entry's rank from two reads, and the entries staged in rank order
        // for coalesced stores.  Each thread takes 16 words per step.
        unsigned *bm = reinterpret_cast<unsigned *>(vals);
        unsigned *pw = reinterpret_cast<unsigned *>(keys);
        const unsigned short *pref = reinterpret_cast<const unsigned short *>(keys);
        const int W16 = (((ncols + 31) >> 5) + 15) & ~15;     // at most 2T
        for (int t = gt; t < W16; t += G) bm[t] = 0u;
        group_sync<WPR>();
#pragma unroll
        for (int s = 0; s < SPT; ++s)
            if (kr[s] != kEmpty) atomicOr(&bm[(kr[s] - lo) >> 5], 1u << ((kr[s] - lo) & 31));
        group_sync<WPR>();
        int run = 0;
        for (int g0 = 0; g0 < W16; g0 += 16 * G) {
            const int w0 = g0 + gt * 16;
            int c[16];
            int pc = 0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                c[q] = w0 < W16 ? __popc(bm[w0 + q]) : 0;
                pc += c[q];
            }
            const int inc = wave_incl_scan(pc);
            if (lane == kWave - 1) s_scan[wg] = inc;
            group_sync<WPR>();
            int wb = 0, tot = 0;
            for (int w = 0; w < WPR; ++w) {
                const int t = s_scan[w];
                if (w < wg) wb += t;
                tot += t;
            }
            if (w0 < W16) {
                unsigned p = (unsigned)(run + wb + inc - pc);
#pragma unroll
                for (int q = 0; q < 16; q += 2) {
                    const unsigned p1 = p + c[q];
                    pw[(w0 >> 1) + (q >> 1)] = p | (p1 << 16);
                    p = p1 + c[q + 1];
                }
            }
            run += tot;
            group_sync<WPR>();
        }
        int rk[SPT];
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            rk[s] = -1;
            if (kr[s] != kEmpty) {
                const int j = kr[s] - lo, w = j >> 5;
                rk[s] = (int)pref[w] + __popc(bm[w] & ((1u << (j & 31)) - 1u));
            }
        }
        group_sync<WPR>();
#pragma unroll
        for (int s = 0; s < SPT; ++s)
            if (rk[s] >= 0 && rk[s] < T) {
                keys[rk[s]] = kr[s];
                vals[rk[s]] = vr[s];
            }
        total = run;
    } else {
        int pos = wbase + incl - cnt;
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            if (kr[s] != kEmpty) {
                keys[pos] = kr[s];
                vals[pos] = vr[s];
                ++pos;
            }
        }
        if constexpr (WPR == 1) {
            if (total <= kWave) {
                // one wave, at most 64 entries: lane l takes entry l, and its
                // rank is the number of smaller columns, counted over the
                // wave's lanes (no sorting network, no LDS round trips)
                wave_sync();
                const int lane = lane_id();
                const int k = lane < total ? keys[lane] : 0x7fffffff;
                const double v = lane < total ? vals[lane] : 0.0;
                int r = 0;
                for (int q = 0; q < total; ++q) r += __builtin_amdgcn_readlane(k, q) < k;
                wave_sync();
                if (lane < total) {
                    keys[r] = k;
                    vals[r] = v;
                }
                wave_sync();
                return total;
            }
        }
        const int n2 = total <= 1 ? 1 : (1 << ceil_log2(total));
        for (int t = total + gt; t < n2; t += G) keys[t] = 0x7fffffff;
        group_sync<WPR>();
        group_bitonic<double, WPR>(keys, vals, n2, gt);
    }
    group_sync<WPR>();
    return total;
}

// Write-back of an order-preserving table (the paper's Write-back Phase,
// whose insertion sort finishes the order of a semi-sorted table).  kr/vr
// hold each thread's SPT slots; home(j) = j >> shift; D is the longest probe
// distance.  The occupied slots are compacted in "unwrapped" slot order:
// entries at or after their home slot by slot, then those that wrapped past
// the table's end.  In that order an entry lies at most D places from its
// place in column order (two entries can be out of order only if both lie
// within D slots of the lower one's home), so its rank is its position
// corrected by the entries within D places on either side that belong on
// its other side: the bounded form of insertion sort, one entry per thread.
// Leaves the entries in column order at the front of keys/vals; returns
// their number.  s_scan holds WPR + 1 ints.
template <int T, int WPR, int SPT>
__device__ __forceinline__ int order_row_entries_ord(const int (&kr)[SPT], const double (&vr)[SPT], int *keys,
                                                     double *vals, int *s_scan, int gt, int shift, int D)
{
    constexpr int G = WPR * kWave;
    const int lane = lane_id(), wg = gt / kWave;
    int packed = 0;                                   // non-wrapped | wrapped << 16
#pragma unroll
    for (int s = 0; s < SPT; ++s)
        if (kr[s] != kEmpty) packed += (gt * SPT + s) >= (int)((unsigned)kr[s] >> shift) ? 1 : (1 << 16);
    const int incl = wave_incl_scan(packed);
    group_sync<WPR>();
    if (lane == kWave - 1) s_scan[wg] = incl;
    group_sync<WPR>();
    int base = 0, tot = 0;
    for (int w = 0; w < WPR; ++w) {
        const int t = s_scan[w];
        if (w < wg) base += t;
        tot += t;
    }
    const int n0 = tot & 0xffff, total = n0 + (tot >> 16);
    const int ex = base + incl - packed;
    int p0 = ex & 0xffff, p1 = n0 + (ex >> 16);
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        if (kr[s] == kEmpty) continue;
        const int at = (gt * SPT + s) >= (int)((unsigned)kr[s] >> shift) ? p0++ : p1++;
        keys[at] = kr[s];
        vals[at] = vr[s];
    }
    group_sync<WPR>();
    int xk[SPT], rk[SPT];
    double xv[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
        const int i = gt + q * G;
        rk[q] = -1;
        if (i < total) {
            const int x = keys[i];
            int r = i;
            for (int d = 1; d <= D; ++d) {
                if (i - d >= 0 && keys[i - d] > x) --r;
                if (i + d < total && keys[i + d] < x) ++r;
            }
            xk[q] = x;
            xv[q] = vals[i];
            rk[q] = r;
        }
    }
    group_sync<WPR>();
#pragma unroll
    for (int q = 0; q < SPT; ++q)
        if (rk[q] >= 0 && rk[q] < T) {
            keys[rk[q]] = xk[q];
            vals[rk[q]] = xv[q];
        }
    group_sync<WPR>();
    return total;
}

// Numeric pass of one light row by a group of WPR waves (steps a5 and a7):
// the products of the row's A entries [e0, e1) times B merged in an LDS
// tag/value table of 2^LOGT slots, then written in column order at C's
// offset rb (nc entries expected).  When B has
// at most 64 * 2^LOGT columns the order comes from ranks in an occupancy
// bitmap over all of B's columns, built in the table's own LDS once its
// entries are in registers (no sort); otherwise the occupied slots are
// compacted and sorted (bitonic).
// HASH selects the table's hash: 0 = multiplicative, 1 = order-preserving
// (home slot j >> shift, shift = ceil(log2 ncols) - LOGT, at least 0, with
// the bounded insertion write-back of order_row_entries_ord; s_maxd is the
// group's LDS word for the longest probe).
template <typename V, int LOGT, int WPR, int HASH = 0>
__device__ __forceinline__ void num_row(int e0, int e1, const int *__restrict__ Acol, const V *__restrict__ Aval,
                                        const int *__restrict__ Brp, const int *__restrict__ Bcol,
                                        const V *__restrict__ Bval, long long rb, int nc, bool active, int gt,
                                        int *keys, double *vals, EnumScratch<V, WPR * kWave> &en, int *s_scan,
                                        int *__restrict__ Ccol, V *__restrict__ Cval, int ncols, int *err,
                                        int *s_maxd = nullptr)
{
    constexpr int T = 1 << LOGT;
    constexpr int G = WPR * kWave;
    constexpr int SPT = T / G;          // slots per thread in the compaction
    static_assert(SPT >= 1, "table smaller than its group");
    const int lane = lane_id(), wg = gt / kWave;
    const int lc = ceil_log2(ncols);
    const int shift = lc > LOGT ? lc - LOGT : 0;
    for (int t = gt; t < T; t += G) {
        keys[t] = kEmpty;
        vals[t] = 0.0;
    }
    if constexpr (HASH == 1)
        if (gt == 0) *s_maxd = 0;
    group_sync<WPR>();
    if (active) {
        auto get = [&](int e, int &bs, int &bl, V &a) {
            const int k = Acol[e];
            bs = Brp[k];
            bl = Brp[k + 1] - bs;
            a = Aval[e];
        };
        auto sink = [&](const int (&j)[2], const double (&p)[2], const bool (&ok)[2]) {
            if constexpr (HASH == 1) lds_insert_add_ord_u<2>(keys, vals, LOGT, shift, j, p, ok, s_maxd, err);
            else lds_insert_add_u<2>(keys, vals, LOGT, j, p, ok, err);
        };
        group_products<V, true, G, 2, decltype(get), decltype(sink), true>(e0, e1, gt, en, Bcol, Bval, get, sink);
    }
    group_sync<WPR>();
    if constexpr (HASH == 1) {
        int kr[SPT];
        double vr[SPT];
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            kr[s] = keys[gt * SPT + s];
            vr[s] = vals[gt * SPT + s];
        }
        const int D = *s_maxd;
        const int total = order_row_entries_ord<T, WPR, SPT>(kr, vr, keys, vals, s_scan, gt, shift, D);
        if (active) {
            if (gt == 0 && nc != total) atomicOr(err, kErrCount);
            const int nw = total < nc ? total : nc;
            for (int t = gt; t < nw; t += G) {
                store_c(&Ccol[rb + t], keys[t]);
                store_c(&Cval[rb + t], (V)vals[t]);
            }
        }
        return;
    }
    // compaction of the occupied slots to the front of the table
    int kr[SPT];
    double vr[SPT];
    int cnt = 0;
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        kr[s] = keys[gt * SPT + s];
        vr[s] = vals[gt * SPT + s];
        cnt += kr[s] != kEmpty;
    }
    const int incl = wave_incl_scan(cnt);
    if (lane == kWave - 1) s_scan[wg] = incl;
    group_sync<WPR>();
    int wbase = 0, total = 0;
    for (int w = 0; w < WPR; ++w) {
        const int t = s_scan[w];
        if (w < wg) wbase += t;
        total += t;
    }
    order_row_entries<T, WPR, SPT>(kr, vr, keys, vals, s_scan, total, wbase, incl, cnt, ncols, gt);
    if (active) {
        if (gt == 0 && nc != total) atomicOr(err, kErrCount);
        const int nw = total < nc ? total : nc;
        for (int t = gt; t < nw; t += G) {
            store_c(&Ccol[rb + t], keys[t]);
            store_c(&Cval[rb + t], (V)vals[t]);
        }
    }
}

// Light rows: one row per group of WPR waves (RPW groups per block).
template <typename V, int LOGT, int WPR, int RPW, int HASH = 0>
__global__ __launch_bounds__(kWave *WPR *RPW) void k_num_rows(
    const int *__restrict__ Arp, const int *__restrict__ Acol, const V *__restrict__ Aval,
    const int *__restrict__ Brp, const int *__restrict__ Bcol, const V *__restrict__ Bval,
    const int *__restrict__ rows, int nrows, const long long *__restrict__ Crp, int *__restrict__ Ccol,
    V *__restrict__ Cval, int ncols, int *err)
{
    static_assert(RPW == 1 || WPR == 1, "multi-row blocks use one wave per row");
    constexpr int T = 1 << LOGT;
    constexpr int G = WPR * kWave;
    __shared__ int s_keys[RPW][T];
    __shared__ double s_vals[RPW][T];
    __shared__ EnumScratch<V, G> s_en[RPW];
    __shared__ int s_scan[RPW][WPR + 1];
    __shared__ int s_maxd[RPW];
    const int g = threadIdx.x / kWave / WPR;
    const int gt = threadIdx.x - g * G;
    const int r = blockIdx.x * RPW + g;
    const bool active = r < nrows;
    const int row = active ? rows[r] : 0;
    const int e0 = active ? Arp[row] : 0, e1 = active ? Arp[row + 1] : 0;
    const long long rb = active ? Crp[row] : 0;
    const int nc = active ? (int)(Crp[row + 1] - rb) : 0;
    num_row<V, LOGT, WPR, HASH>(e0, e1, Acol, Aval, Brp, Bcol, Bval, rb, nc, active, gt, s_keys[g], s_vals[g],
                                s_en[g], s_scan[g], Ccol, Cval, ncols, err, &s_maxd[g]);
}

// ---------------------------------------------------------------- row scan

// out = exclusive prefix of cnt (int or int64 counts) in three passes over
// blocks of kScanItems entries; out[n] and *total receive the sum.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanItems = kScanThreads * kScanPer;

template <typename TIn>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(long long n, const TIn *__restrict__ cnt,
                                                              long long *__restrict__ bsum)
{
    __shared__ long long s_tmp[kScanThreads / kWave + 1];
    const long long base = (long long)blockIdx.x * kScanItems + threadIdx.x * kScanPer;
    long long s = 0;
#pragma unroll
    for (int t = 0; t < kScanPer; ++t)
        if (base + t < n) s += cnt[base + t];
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

template <typename TIn>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(long long n, const TIn *__restrict__ cnt,
                                                             const long long *__restrict__ boff,
                                                             const long long *__restrict__ total,
                                                             long long *__restrict__ out)
{
    __shared__ long long s_tmp[kScanThreads / kWave + 1];
    const long long base = (long long)blockIdx.x * kScanItems + threadIdx.x * kScanPer;
    long long v[kScanPer];
    long long s = 0;
#pragma unroll
    for (int t = 0; t < kScanPer; ++t) {
        v[t] = base + t < n ? (long long)cnt[base + t] : 0;
        s += v[t];
    }
    long long tot;
    long long run = block_excl_scan<long long, kScanThreads>(s, s_tmp, tot) + boff[blockIdx.x];
#pragma unroll
    for (int t = 0; t < kScanPer; ++t) {
        if (base + t < n) out[base + t] = run;
        run += v[t];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = *total;
}

// ------------------------------------------------------ heavy rows: chunks

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

// Split points of every B row at the chunk boundaries:
// Bsplit[k * (nchunks + 1) + c] = first position of row k with column >= c * kChunkCols.
__global__ __launch_bounds__(256) void k_bsplit(int brows, int nchunks, const int *__restrict__ Brp,
                                                const int *__restrict__ Bcol, int *__restrict__ Bsplit, const int *err)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long per = nchunks + 1;
    if (t >= (long long)brows * per || stopped(err)) return;
    const int k = (int)(t / per), c = (int)(t % per);
    const int b0 = Brp[k], b1 = Brp[k + 1];
    int pos;
    if (c == 0) pos = b0;
    else if (c == nchunks) pos = b1;
    else pos = lower_bound_col(Bcol, b0, b1, c * kChunkCols);
    Bsplit[t] = pos;
}

// Symbolic phase of heavy rows: block (w, h) marks the columns of heavy row h
// that fall in symbolic window w (kSymWinChunks chunks) in an LDS bitmap, then
// stores the number of columns of every chunk (wcnt) and adds them to the
// row's count.  The grid covers hcap heavy rows (the workspace's capacity, a
// host-side bound); the number present, sh->count[kBinHeavy], comes from the
// device, and blocks beyond it return at once.
constexpr int kSymHeavyThreads = 256;

__global__ __launch_bounds__(kSymHeavyThreads) void k_sym_heavy(
    const int *__restrict__ Arp, const int *__restrict__ Acol, const int *__restrict__ Bcol,
    const int *__restrict__ Bsplit, long long per, const int *__restrict__ perm, const BinHdr *sh, int hcap,
    int nchunks, int *__restrict__ wcnt, int *__restrict__ nnzc, const int *err)
{
    constexpr int G = kSymHeavyThreads;
    constexpr int WG = G / kWave;
    constexpr int WORDS = kSymWinChunks * kChunkWords;
    __shared__ unsigned bm[WORDS];
    __shared__ RunScratch<float, G> S;
    // window-major: blocks launched together share one column window of B
    const int w = blockIdx.x / hcap, h = blockIdx.x % hcap;
    if (h >= sh->count[kBinHeavy] || stopped(err)) return;
    const int row = perm[sh->offset[kBinHeavy] + h];
    const int gt = threadIdx.x, lane = lane_id(), wg = gt / kWave;
    const int c0 = w * kSymWinChunks;
    const int c1 = c0 + kSymWinChunks < nchunks ? c0 + kSymWinChunks : nchunks;
    const int lo = c0 * kChunkCols;
    const int *__restrict__ split0 = Bsplit + c0;
    const int *__restrict__ split1 = Bsplit + c1;
    for (int t = gt; t < WORDS; t += G) bm[t] = 0u;
    __syncthreads();
    auto get = [&](int e, int &bs, int &bl, float &) {
        const int k = Acol[e];
        bs = split0[k * per];
        bl = split1[k * per] - bs;
    };
    // all words of the thread's products are read before any is tested, so
    // the reads overlap; most repeated columns then skip the atomic (an OR
    // after a stale read is merely redundant)
    auto sink = [&](const auto &j, const auto &ok) {
        constexpr int N = sizeof(j) / sizeof(j[0]);
        unsigned w[N];
#pragma unroll
        for (int u = 0; u < N; ++u) w[u] = ok[u] ? bm[(j[u] - lo) >> 5] : ~0u;
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const unsigned bit = 1u << ((j[u] - lo) & 31);
            if (!(w[u] & bit)) atomicOr(&bm[(j[u] - lo) >> 5], bit);
        }
    };
    run_products<float, false, G, G, 8, 2, kRun, decltype(get), decltype(sink), true>(
        Arp[row], Arp[row + 1], gt, S, Bcol, (const float *)nullptr, get, sink);
    __syncthreads();
    // per-chunk counts: one wave per chunk
    int local = 0;
    for (int c = wg; c < c1 - c0; c += WG) {
        int pc = 0;
        for (int t = lane; t < kChunkWords; t += kWave) pc += __popc(bm[c * kChunkWords + t]);
        pc = wave_sum(pc);
        if (lane == 0) wcnt[(long long)h * nchunks + c0 + c] = pc;
        local += pc;
    }
    if (lane == 0 && local) atomicAdd(&nnzc[row], local);
}

// Exclusive prefix of the chunk counts of every heavy row (row-relative output
// offsets of the chunks); one wave per heavy row, 64 chunks per step
// (coalesced).
__global__ __launch_bounds__(256) void k_chunk_prefix(const BinHdr *sh, int nchunks, const int *__restrict__ wcnt,
                                                      int *__restrict__ woff, const int *err)
{
    const int h = blockIdx.x * 4 + threadIdx.x / kWave;
    if (h >= sh->count[kBinHeavy] || stopped(err)) return;
    const int lane = lane_id();
    const long long base = (long long)h * nchunks;
    int run = 0;
    for (int c0 = 0; c0 < nchunks; c0 += kWave) {
        const int c = c0 + lane;
        const int v = c < nchunks ? wcnt[base + c] : 0;
        const int incl = wave_incl_scan(v);
        if (c < nchunks) woff[base + c] = run + incl - v;
        run += __shfl(incl, kWave - 1, kWave);
    }
}

// Cuts every heavy row into segments (one thread per heavy row): a chunk
// with more than kSegCap columns is a dense segment of its own; otherwise
// consecutive chunks are merged while the count stays <= kSegMerge and the
// span <= kSegMaxSpan chunks (a single chunk of up to kSegCap entries is a
// segment of its own: smaller merged segments keep more of them in the
// 1024-slot tables, which fit more blocks per CU).  Pass 0 counts segments per block and bin;
// pass 1 writes them at offset[bin] + block base + rank in block.
__device__ __forceinline__ int seg_bin(int count, bool dense)
{
    return dense ? kSegDense : (count <= 128 ? 0 : (count <= 700 ? 1 : 2));
}

template <typename F>
__device__ __forceinline__ void plan_row_segments(const int *__restrict__ wc, int nchunks, F emit)
{
    int c = 0;
    while (c < nchunks) {
        const int n0 = wc[c];
        if (n0 == 0) { ++c; continue; }
        if (n0 > kSegCap) { emit(c, c + 1, n0, true); ++c; continue; }
        const int start = c;
        int sum = 0, last = c;
        while (c < nchunks && c - start < kSegMaxSpan) {
            const int n = wc[c];
            if (n > kSegCap || (sum + n > kSegMerge && sum > 0)) break;
            sum += n;
            if (n) last = c;
            ++c;
        }
        emit(start, last + 1, sum, false);
        c = last + 1;
    }
}

// Segments are laid out bin by bin and, within a bin, chunk by chunk (by
// their first chunk): blocks launched together then work on the same column
// slice of B, which stays in L2.  Pass 0 counts segments per (bin, chunk) in
// hist; k_seg_scan turns the counts into offsets (and cursors); pass 1 writes
// every segment at its (bin, chunk) cursor.  Blocks aggregate their counts
// in LDS (one global atomic per block and group) when the kSegBins x nchunks
// histogram fits kSegPlanLds entries.
constexpr int kSegPlanLds = 4096;

__global__ __launch_bounds__(256) void k_seg_plan(int pass, const BinHdr *bh, const int *__restrict__ perm,
                                                  int nchunks, const int *__restrict__ wcnt,
                                                  const int *__restrict__ woff, const int *__restrict__ Arp,
                                                  const long long *__restrict__ Crp, int *__restrict__ hist,
                                                  SegHdr *sh, Seg *__restrict__ segs, const int *err)
{
    if (stopped(err)) return;
    const int nheavy = bh->count[kBinHeavy];
    const int *__restrict__ heavy_rows = perm + bh->offset[kBinHeavy];
    __shared__ unsigned long long s_nnz[kSegBins];
    __shared__ int s_cnt[kSegPlanLds];
    const int cells = kSegBins * nchunks;
    const bool local = cells <= kSegPlanLds;
    if (threadIdx.x < kSegBins) s_nnz[threadIdx.x] = 0;
    if (local)
        for (int t = threadIdx.x; t < cells; t += 256) s_cnt[t] = 0;
    __syncthreads();
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    const int *wc = wcnt + (long long)h * nchunks;
    // count this block's segments per (bin, chunk)
    if (h < nheavy) {
        long long lnnz[kSegBins] = {0, 0, 0, 0};
        plan_row_segments(wc, nchunks, [&](int a, int, int n, bool dense) {
            const int b = seg_bin(n, dense);
            if (pass == 0) {
                if (local) atomicAdd(&s_cnt[b * nchunks + a], 1);
                else atomicAdd(&hist[(long long)b * nchunks + a], 1);
                lnnz[b] += n;
            } else if (local) {
                atomicAdd(&s_cnt[b * nchunks + a], 1);
            }
        });
        if (pass == 0)
            for (int b = 0; b < kSegBins; ++b)
                if (lnnz[b]) atomicAdd(&s_nnz[b], (unsigned long long)lnnz[b]);
    }
    __syncthreads();
    if (pass == 0) {
        if (local)
            for (int t = threadIdx.x; t < cells; t += 256)
                if (s_cnt[t]) atomicAdd(&hist[t], s_cnt[t]);
        if (threadIdx.x < kSegBins && s_nnz[threadIdx.x])
            atomicAdd((unsigned long long *)&sh->nnz[threadIdx.x], s_nnz[threadIdx.x]);
        return;
    }
    // pass 1: reserve this block's range of every group, then place
    if (local)
        for (int t = threadIdx.x; t < cells; t += 256)
            s_cnt[t] = s_cnt[t] ? atomicAdd(&hist[t], s_cnt[t]) : 0;
    __syncthreads();
    if (h < nheavy) {
        const int row = heavy_rows[h];
        const int e0 = Arp[row], e1 = Arp[row + 1];
        const long long rb = Crp[row];
        const int *wo = woff + (long long)h * nchunks;
        plan_row_segments(wc, nchunks, [&](int a, int b, int n, bool dense) {
            const int bin = seg_bin(n, dense);
            const int cell = bin * nchunks + a;
            const int pos = local ? atomicAdd(&s_cnt[cell], 1) : atomicAdd(&hist[cell], 1);
            segs[pos] = Seg{row, e0, e1, a, b, n, rb + wo[a]};
        });
    }
}

// Offsets of the segment bins and of every (bin, chunk) group; hist becomes
// the write cursor of each group (one wave).
__global__ __launch_bounds__(kWave) void k_seg_scan(int nchunks, int *__restrict__ hist, SegHdr *sh, const int *err)
{
    if (stopped(err)) return;
    const int lane = lane_id();
    int run = 0;
    for (int b = 0; b < kSegBins; ++b) {
        if (lane == 0) sh->offset[b] = run;
        const int start = run;
        for (int c0 = 0; c0 < nchunks; c0 += kWave) {
            const int c = c0 + lane;
            const long long at = (long long)b * nchunks + c;
            const int v = c < nchunks ? hist[at] : 0;
            const int incl = wave_incl_scan(v);
            if (c < nchunks) hist[at] = run + incl - v;
            run += __shfl(incl, kWave - 1, kWave);
        }
        if (lane == 0) sh->count[b] = run - start;
    }
    if (lane == 0) sh->offset[kSegBins] = run;
}

// Hashed segment of a heavy row: products of the row whose columns lie in
// chunks [c0, c1) merged in an LDS table of 2^LOGT slots; entries ranked by
// an occupancy bitmap of the segment's columns (built in the table's own
// storage once the entries are in registers, so the block needs no other
// LDS and more blocks fit a CU), staged in column order and copied out with
// coalesced stores.
template <typename V, int LOGT, int THREADS>
__global__ __launch_bounds__(THREADS) void k_num_seg(
    const int *__restrict__ Arp, const int *__restrict__ Acol, const V *__restrict__ Aval,
    const int *__restrict__ Bcol, const V *__restrict__ Bval, const int *__restrict__ Bsplit, long long per,
    const int *__restrict__ heavy_rows, const Seg *__restrict__ segs, int nchunks,
    const int *__restrict__ woff, const long long *__restrict__ Crp, int *__restrict__ Ccol,
    V *__restrict__ Cval, int *err)
{
    constexpr int T = 1 << LOGT;
    constexpr int SPT = T / THREADS;
    static_assert(SPT >= 1, "table smaller than the block");
    constexpr int WPR = THREADS / kWave;
    __shared__ int keys[T];
    __shared__ double vals[T];
    __shared__ EnumScratch<V, THREADS> S;
    __shared__ int s_scan[WPR + 1];
    const Seg sg = segs[blockIdx.x];
    const int gt = threadIdx.x;
    const int lo = sg.c0 * kChunkCols;
    const int *__restrict__ split0 = Bsplit + sg.c0;
    const int *__restrict__ split1 = Bsplit + sg.c1;
    for (int t = gt; t < T; t += THREADS) {
        keys[t] = kEmpty;
        vals[t] = 0.0;
    }
    __syncthreads();
    auto get = [&](int e, int &bs, int &bl, V &a) {
        const int k = Acol[e];
        bs = split0[k * per];
        bl = split1[k * per] - bs;
        a = Aval[e];
    };
    // one product per thread in flight: the segment kernels are bound by how
    // many blocks fit a CU, and fewer registers per thread let more in
    auto sink = [&](const int (&j)[1], const double (&p)[1], const bool (&ok)[1]) {
        lds_insert_add_u<1>(keys, vals, LOGT, j, p, ok, err);
    };
    group_products<V, true, THREADS, 1, decltype(get), decltype(sink), true>(sg.e0, sg.e1, gt, S, Bcol, Bval, get,
                                                                            sink);
    __syncthreads();
    int kr[SPT];
    double vr[SPT];
    int cnt = 0;
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        kr[s] = keys[gt * SPT + s];
        vr[s] = vals[gt * SPT + s];
        cnt += kr[s] != kEmpty;
    }
    int incl = 0, wbase = 0, total = 0;
    if constexpr (64 * T < kSegMaxSpan * kChunkCols) {
        // a segment can be too wide for the bitmap ranks, and the sort that
        // takes it then needs each thread's place among the entries
        const int lane = lane_id(), wg = gt / kWave;
        incl = wave_incl_scan(cnt);
        if (lane == kWave - 1) s_scan[wg] = incl;
        __syncthreads();
        for (int w = 0; w < WPR; ++w) {
            const int t = s_scan[w];
            if (w < wg) wbase += t;
            total += t;
        }
    }
    total = order_row_entries<T, WPR, SPT>(kr, vr, keys, vals, s_scan, total, wbase, incl, cnt,
                                           (sg.c1 - sg.c0) * kChunkCols, gt, lo);
    if (gt == 0 && total != sg.count) atomicOr(err, kErrCount);
    const long long out0 = sg.out;
    const int n = total < sg.count ? total : sg.count;
    for (int t = gt; t < n; t += THREADS) {
        store_c(&Ccol[out0 + t], keys[t]);
        store_c(&Cval[out0 + t], (V)vals[t]);
    }
}

constexpr long long kNegZeroBits = (long long)0x8000000000000000ULL;

// A slot of a dense window was reached by a product when its sum is no
// longer the bit pattern of -0.0 (the window starts at -0.0 and every
// product is added as p + 0.0).
__device__ __forceinline__ bool reached(double v) { return __double_as_longlong(v) != kNegZeroBits; }

// Mask of the lanes of the wave for which p holds (a compare straight into
// a scalar register pair, with no 0/1 select in between).
__device__ __forceinline__ unsigned long long wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Number of lanes below this one whose bit is set in m.
__device__ __forceinline__ int lanes_below(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Stores the entries a wave has ranked in its ROUNDS x 64 slots of a dense
// window: slot r * 64 + lane holds column col0 + r * 64 + lane and value
// vr[r], occupied where reached(vr[r]); msk[r] = wave_ballot(reached(vr[r])).  The first n of them,
// in column order, go to C[out, out + n): staged in the wave's own LDS slots
// (whose values are already in registers) and copied with consecutive lanes
// on consecutive addresses, so stores cover whole cache lines.  FP32 stages
// (column, value) pairs in one pass, FP64 columns and then values.  Every
// lane of the wave calls it; the slots are left dirty.
template <typename V, int ROUNDS>
__device__ __forceinline__ void wave_store_ranked(const double (&vr)[ROUNDS], const unsigned long long (&msk)[ROUNDS],
                                                  double *slots, int col0, long long out, int n,
                                                  int *__restrict__ Ccol, V *__restrict__ Cval)
{
    const int lane = lane_id();
    int lr = 0;
    if constexpr (sizeof(V) == 4) {
        int2 *st = reinterpret_cast<int2 *>(slots);
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            if (reached(vr[r]))
                st[lr + lanes_below(msk[r])] = make_int2(col0 + r * kWave + lane, __float_as_int((float)vr[r]));
            lr += __popcll(msk[r]);
        }
        wave_sync();
        for (int k = lane; k < n; k += kWave) {
            const int2 e = st[k];
            store_c(&Ccol[out + k], e.x);
            store_c(&Cval[out + k], (V)__int_as_float(e.y));
        }
    } else {
        int *st_col = reinterpret_cast<int *>(slots);
        V *st_val = reinterpret_cast<V *>(slots);
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            if (reached(vr[r])) st_col[lr + lanes_below(msk[r])] = col0 + r * kWave + lane;
            lr += __popcll(msk[r]);
        }
        wave_sync();
        for (int k = lane; k < n; k += kWave) store_c(&Ccol[out + k], st_col[k]);
        wave_sync();
        lr = 0;
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            if (reached(vr[r])) st_val[lr + lanes_below(msk[r])] = (V)vr[r];
            lr += __popcll(msk[r]);
        }
        wave_sync();
        for (int k = lane; k < n; k += kWave) store_c(&Cval[out + k], st_val[k]);
    }
    wave_sync();
}

// Dense chunk of a heavy row: products whose columns lie in chunk c0 added
// directly into an LDS array of doubles indexed by column; each wave then
// ranks its own 1024 columns with ballots, stages its entries in column
// order in those same LDS slots and copies them to C with whole-line stores.
// Occupancy needs no bitmap: the array starts at -0.0 and every product is
// added as p + 0.0, which is never -0.0, so a column was reached exactly when
// its sum is no longer the bit pattern of -0.0 (a sum of terms that are not
// -0.0 is never -0.0 under round-to-nearest, even when they cancel).  The
// kernel is persistent: a grid that fills the GPU once takes the dense chunks
// from a global queue (one atomic per `claim` chunks), so that long and
// short chunks balance across CUs, and each wave puts -0.0 back in its slots once its
// entries are out, so the array is ready for the next chunk without a
// separate clearing pass.
constexpr int kDenseThreads = 512;
// dense chunks a block claims with one atomic on the queue when every block
// has many to do (one atomic per chunk from every resident block serialises
// on the counter); one at a time otherwise, for the balance of the tail
constexpr int kDenseClaim = 4;
constexpr int kDenseClaimMinPerBlock = 256;

template <typename V>
__global__ __launch_bounds__(kDenseThreads) void k_num_dense(
    const int *__restrict__ Arp, const int *__restrict__ Acol, const V *__restrict__ Aval,
    const int *__restrict__ Bcol, const V *__restrict__ Bval, const int *__restrict__ Bsplit, long long per,
    const int *__restrict__ heavy_rows, const Seg *__restrict__ segs, int nchunks,
    const int *__restrict__ woff, const long long *__restrict__ Crp, int *__restrict__ Ccol,
    V *__restrict__ Cval, int *err, int nseg, int *queue, int claim)
{
    constexpr int NW = kDenseThreads / kWave;
    constexpr int CPW = kChunkCols / NW;              // columns ranked by each wave
    constexpr int ROUNDS = CPW / kWave;
    extern __shared__ __align__(16) unsigned char s_raw[];
    double *acc = (double *)s_raw;                      // [kChunkCols]
    __shared__ EnumScratch<V, kDenseThreads> S;
    __shared__ int s_wt[NW];
    __shared__ int s_next;
    const int gt = threadIdx.x, lane = lane_id(), wg = gt / kWave;
    for (int t = gt; t < kChunkCols; t += kDenseThreads) acc[t] = -0.0;
    for (;;) {
    if (gt == 0) s_next = atomicAdd(queue, claim);
    __syncthreads();                                    // also: the previous chunk is fully written
    const int first = s_next;
    if (first >= nseg) break;
    const int last = first + claim < nseg ? first + claim : nseg;
    for (int t = first; t < last; ++t) {
    const Seg sg = segs[t];
    const int lo = sg.c0 * kChunkCols;
    const int *__restrict__ split0 = Bsplit + sg.c0;
    const int *__restrict__ split1 = split0 + 1;
    auto get = [&](int e, int &bs, int &bl, V &a) {
        const int k = Acol[e];
        bs = split0[k * per];
        bl = split1[k * per] - bs;
        a = Aval[e];
    };
    auto sink = [&](int j, double p) { atomicAdd(&acc[j - lo], p + 0.0); };
    group_products<V, true, kDenseThreads, 2, decltype(get), decltype(sink), false, true>(sg.e0, sg.e1, gt, S, Bcol,
                                                                                          Bval, get, sink);
    __syncthreads();
    double vr[ROUNDS];
    unsigned long long msk[ROUNDS];
    int wcount = 0;
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        vr[r] = acc[wg * CPW + r * kWave + lane];
        msk[r] = wave_ballot(reached(vr[r]));
        wcount += __popcll(msk[r]);
    }
    if (lane == 0) s_wt[wg] = wcount;
    __syncthreads();
    int run = 0, tot = 0;
    for (int w = 0; w < NW; ++w) {
        const int c = s_wt[w];
        if (w < wg) run += c;
        tot += c;
    }
    if (gt == 0 && tot != sg.count) atomicOr(err, kErrCount);
    const int n = wcount < sg.count - run ? wcount : (sg.count - run > 0 ? sg.count - run : 0);
    wave_store_ranked<V, ROUNDS>(vr, msk, acc + wg * CPW, lo + wg * CPW, sg.out + run, n, Ccol, Cval);
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) acc[wg * CPW + r * kWave + lane] = -0.0;   // cleared for the next chunk
    __syncthreads();                                    // s_wt and s_next are reused
    }
    }
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

constexpr int kGlobalThreads = 1024;

// Symbolic count of one heavy row in global mode by a whole block: the row's
// columns are inserted in its global key table of next_pow2(2 cap) slots
// (device-scope CAS; the table must hold kEmpty) and counted into *out.
__device__ __forceinline__ void sym_global_row(const int *__restrict__ Arp, const int *__restrict__ Acol,
                                               const int *__restrict__ Brp, const int *__restrict__ Bcol, int arow,
                                               int cap, int *keys, EnumScratch<float, kGlobalThreads> &S, int *s_cnt,
                                               int *out, int *err)
{
    const int logT = gtable_log2(cap);
    const unsigned mask = (1u << logT) - 1;
    if (threadIdx.x == 0) *s_cnt = 0;
    int mine = 0;
    group_products<float, false, kGlobalThreads, 2>(
        Arp[arow], Arp[arow + 1], threadIdx.x, S, Bcol, (const float *)nullptr,
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
    if (lane_id() == 0 && mine) atomicAdd(s_cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) *out = *s_cnt;
}

// Symbolic phase of heavy rows in global mode: one block per row.
__global__ __launch_bounds__(kGlobalThreads) void k_sym_global(
    const int *__restrict__ Arp, const int *__restrict__ Acol, const int *__restrict__ Brp,
    const int *__restrict__ Bcol, const int *__restrict__ rows, const int *__restrict__ cap,
    const long long *__restrict__ goff, long long gbase, int *gkeys, int *__restrict__ nnzc, int *err)
{
    __shared__ EnumScratch<float, kGlobalThreads> S;
    __shared__ int s_cnt;
    const int row = rows[blockIdx.x];
    sym_global_row(Arp, Acol, Brp, Bcol, row, cap[row], gkeys + (goff[blockIdx.x] - gbase), S, &s_cnt, &nnzc[row],
                   err);
}

// Numeric pass of one heavy row in global mode by a whole block: clears the
// row's global tag/value table, merges the row's products into it with
// device-scope CAS and atomic add (FP64 values: the sum is rounded to the
// output type once, at write-out), then writes the entries in column order
// at C's row `crow`.  Every slot the row claims is appended to the row's
// touched-slot list (`touched`, nc entries: the paper's third version keeps
// its tags in dense arrays with an offset array for the same purpose), so
// the write-out reads the row's nc entries instead of scanning all T >= 2 nc
// slots of its table: per window of kGlobalRankBits columns, the listed
// entries of the window are marked in an LDS bitmap (s_bm, the block's
// dynamic LDS), ranked by its popcount prefix and stored.
constexpr int kGlobalRankBits = 1 << 19;

template <typename V>
struct GlobalNumLds {
    EnumScratch<V, kGlobalThreads> S;
    long long tmp[kGlobalThreads / kWave + 1];
    int base[kGlobalThreads];
    int ntouched;
};

template <typename V>
__device__ __forceinline__ void num_global_row(const int *__restrict__ Arp, const int *__restrict__ Acol,
                                               const V *__restrict__ Aval, const int *__restrict__ Brp,
                                               const int *__restrict__ Bcol, const V *__restrict__ Bval, int arow,
                                               long long crow, int ncols, int *keys, double *vals, int *touched,
                                               GlobalNumLds<V> &L, unsigned *s_bm, const long long *__restrict__ Crp,
                                               int *__restrict__ Ccol, V *__restrict__ Cval, int *err)
{
    constexpr int WORDS = kGlobalRankBits / 32;
    constexpr int WPT = WORDS / kGlobalThreads;
    const long long rb = Crp[crow];
    const int nc = (int)(Crp[crow + 1] - rb);
    const int logT = gtable_log2(nc);
    const int T = 1 << logT;
    const unsigned mask = (unsigned)T - 1;
    for (int t = threadIdx.x; t < T; t += kGlobalThreads) {
        keys[t] = kEmpty;
        vals[t] = 0.0;
    }
    if (threadIdx.x == 0) L.ntouched = 0;
    __threadfence();
    __syncthreads();
    group_products<V, true, kGlobalThreads, 2>(
        Arp[arow], Arp[arow + 1], threadIdx.x, L.S, Bcol, Bval,
        [&](int e, int &bs, int &bl, V &a) {
            const int k = Acol[e];
            bs = Brp[k];
            bl = Brp[k + 1] - bs;
            a = Aval[e];
        },
        [&](int j, double p) {
            unsigned hh = slot_of(j, logT);
            for (unsigned probe = 0; probe <= mask; ++probe) {
                int cur = gload(&keys[hh]);
                if (cur == kEmpty) {
                    int old = atomicCAS(&keys[hh], kEmpty, j);
                    if (old == kEmpty) {                  // claimed: list the slot
                        const int at = atomicAdd(&L.ntouched, 1);
                        if (at < nc) touched[at] = (int)hh;
                    }
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
    const int nt = L.ntouched < nc ? L.ntouched : nc;
    long long done = 0;
    for (int lo = 0; lo < ncols; lo += kGlobalRankBits) {
        const int hi = lo + kGlobalRankBits < ncols ? lo + kGlobalRankBits : ncols;
        for (int t = threadIdx.x; t < WORDS; t += kGlobalThreads) s_bm[t] = 0u;
        __syncthreads();
        for (int t = threadIdx.x; t < nt; t += kGlobalThreads) {
            const int j = gload(&keys[touched[t]]);
            if (j >= lo && j < hi) atomicOr(&s_bm[(j - lo) >> 5], 1u << ((j - lo) & 31));
        }
        __syncthreads();
        int pc = 0;
        for (int q = 0; q < WPT; ++q) pc += __popc(s_bm[threadIdx.x * WPT + q]);
        long long tot;
        const long long ex = block_excl_scan<long long, kGlobalThreads>((long long)pc, L.tmp, tot);
        L.base[threadIdx.x] = (int)ex;
        __syncthreads();
        for (int t = threadIdx.x; t < nt; t += kGlobalThreads) {
            const int slot = touched[t];
            const int j = gload(&keys[slot]);
            if (j < lo || j >= hi) continue;
            const int jl = j - lo, wd = jl >> 5, owner = wd / WPT;
            int rank = L.base[owner];
            for (int q = owner * WPT; q < wd; ++q) rank += __popc(s_bm[q]);
            rank += __popc(s_bm[wd] & ((1u << (jl & 31)) - 1u));
            const long long pos = done + rank;
            if (pos < nc) {
                store_c(&Ccol[rb + pos], j);
                store_c(&Cval[rb + pos], (V)gload_v(&vals[slot]));
            }
        }
        done += tot;
        __syncthreads();
        if (done >= nt) break;                    // every listed entry is out
    }
    if (threadIdx.x == 0 && (done != nc || L.ntouched != nc)) atomicOr(err, kErrCount);
}

// Numeric phase of heavy rows in global mode: one block per row (the row's
// table and touched-slot list start at the same offset of the pool's key,
// value and list arrays).
template <typename V>
__global__ __launch_bounds__(kGlobalThreads) void k_num_global(
    const int *__restrict__ Arp, const int *__restrict__ Acol, const V *__restrict__ Aval,
    const int *__restrict__ Brp, const int *__restrict__ Bcol, const V *__restrict__ Bval,
    const int *__restrict__ rows, int ncols, const long long *__restrict__ goff, long long gbase, int *gkeys,
    double *gvals, int *gtouch, const long long *__restrict__ Crp, int *__restrict__ Ccol, V *__restrict__ Cval,
    int *err)
{
    extern __shared__ unsigned s_bm[];                     // [kGlobalRankBits / 32]
    __shared__ GlobalNumLds<V> L;
    const int row = rows[blockIdx.x];
    const long long at = goff[blockIdx.x] - gbase;
    num_global_row<V>(Arp, Acol, Aval, Brp, Bcol, Bval, row, row, ncols, gkeys + at, gvals + at, gtouch + at, L, s_bm,
                      Crp, Ccol, Cval, err);
}

}  // namespace smash
