// smash_fused.hpp -- the fused single pass for rows the learned predictor
// sizes into LDS.
//
// A row whose predicted capacity fits an LDS table is hashed, counted,
// sorted and staged in one kernel, with no symbolic pass: the table has
// next_pow2(2 * capacity) slots, and the row is accepted when its distinct
// columns fit the capacity.  A row that does not fit (the prediction was
// too small) is marked and handed to the exact two-phase path, as are rows
// predicted too large for LDS.  After the row-pointer scan the staged rows
// are copied to their final offsets.
#pragma once

#include <hip/hip_runtime.h>

#include "smash_kernels.hpp"

namespace smash {

// Fused bin of a row: LDS bin of its predicted capacity when
// 0 < ub_i and cap_i <= fused_max, else kBinEmpty (not fused).
__global__ __launch_bounds__(256) void k_fused_bins(int m, const long long *__restrict__ ub,
                                                    const int *__restrict__ cap_pred, int fused_max,
                                                    unsigned char *__restrict__ fbin, int *__restrict__ fcap,
                                                    const int *err)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m || stopped(err)) return;
    const int c = cap_pred[i];
    const bool fused = ub[i] > 0 && c > 0 && c <= fused_max;
    fbin[i] = (unsigned char)(fused ? lds_bin(c) : kBinEmpty);
    fcap[i] = fused ? c : 0;
}

// Like lds_insert_add_u, but a row stops inserting once it holds more
// distinct columns than its capacity (*ndist counts them, *abort is
// raised): the table then stays at most about half full (plus one wave
// step of keys), so probes stay short however wrong the prediction was.
// The wave's new keys are counted with ballots and added to *ndist by one
// lane (one LDS atomic per wave step instead of one per new key, all on
// the same address).  Every lane of the wave calls it.
template <int U>
__device__ __forceinline__ void lds_bounded_insert_add_u(int *keys, double *vals, int logT, const int (&j)[U],
                                                         const double (&p)[U], const bool (&okin)[U], int cap,
                                                         int *ndist, int *abort)
{
    if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return;
    const unsigned mask = (1u << logT) - 1;
    unsigned h[U];
    int old[U];
#pragma unroll
    for (int u = 0; u < U; ++u) h[u] = slot_of(j[u], logT);
#pragma unroll
    for (int u = 0; u < U; ++u) old[u] = okin[u] ? atomicCAS(&keys[h[u]], kEmpty, j[u]) : j[u];
    bool fresh[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        fresh[u] = false;
        if (!okin[u]) continue;
        unsigned hh = h[u];
        int cur = old[u];
        for (unsigned probe = 0;; ++probe) {
            if (cur == kEmpty) {                    // claimed a new slot
                atomicAdd(&vals[hh], p[u]);
                fresh[u] = true;
                break;
            }
            if (cur == j[u]) {
                atomicAdd(&vals[hh], p[u]);
                break;
            }
            if (probe >= mask) {                    // table full: only after a wrong prediction
                atomicExch(abort, 1);
                break;
            }
            hh = (hh + 1) & mask;
            cur = atomicCAS(&keys[hh], kEmpty, j[u]);
        }
    }
    int added = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) added += __popcll(__ballot(fresh[u]));
    if (lane_id() == 0 && added > 0 && atomicAdd(ndist, added) + added > cap) atomicExch(abort, 1);
}

// Fused rows: products merged in an LDS table of 2^LOGT slots; a row whose
// columns fit its capacity is put in column order (bitmap ranks or sort, as
// for the rows of the two-phase path) and written to the staging area at
// stage_off[row] (status 1, nnzc = count); otherwise status 0 and the row is
// left to the two-phase path.  Rows of the stage that would end beyond
// stage_cap entries are left to the two-phase path too.  Persistent grid
// over the bin's rows (perm + h->offset[bin], h->count[bin] from the
// device), like k_sym_rows.
template <typename V, int LOGT, int WPR, int RPW>
__global__ __launch_bounds__(kWave *WPR *RPW) void k_fused_rows(
    const int *__restrict__ Arp, const int *__restrict__ Acol, const V *__restrict__ Aval,
    const int *__restrict__ Brp, const int *__restrict__ Bcol, const V *__restrict__ Bval,
    const int *__restrict__ perm, const BinHdr *h, int bin, const int *__restrict__ fcap,
    const long long *__restrict__ stage_off, long long stage_cap, int *__restrict__ scol, V *__restrict__ sval,
    int *__restrict__ nnzc, unsigned char *__restrict__ status, int ncols, const int *err)
{
    static_assert(RPW == 1 || WPR == 1, "multi-row blocks use one wave per row");
    constexpr int T = 1 << LOGT;
    constexpr int G = WPR * kWave;
    constexpr int SPT = T / G;
    if (stopped(err)) return;
    __shared__ int s_keys[RPW][T];
    __shared__ double s_vals[RPW][T];
    __shared__ EnumScratch<V, G> s_en[RPW];
    __shared__ int s_scan[RPW][WPR + 1];
    __shared__ int s_full[RPW];
    __shared__ int s_ndist[RPW];
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const int g = wave / WPR, wg = wave % WPR;
    const int gt = threadIdx.x - g * G;
    const int nrows = h->count[bin];
    const int *rows = perm + h->offset[bin];
    for (int r0 = blockIdx.x * RPW; r0 < nrows; r0 += gridDim.x * RPW) {
    const int r = r0 + g;
    const bool active = r < nrows;
    const int row = active ? rows[r] : 0;
    int *keys = s_keys[g];
    double *vals = s_vals[g];
    for (int t = gt; t < T; t += G) {
        keys[t] = kEmpty;
        vals[t] = 0.0;
    }
    if (gt == 0) {
        s_full[g] = 0;
        s_ndist[g] = 0;
    }
    const int cap = active ? fcap[row] : 0;
    group_sync<WPR>();
    if (active) {
        auto get = [&](int e, int &bs, int &bl, V &a) {
            const int k = Acol[e];
            bs = Brp[k];
            bl = Brp[k + 1] - bs;
            a = Aval[e];
        };
        auto sink = [&](const int (&j)[2], const double (&p)[2], const bool (&ok)[2]) {
            lds_bounded_insert_add_u<2>(keys, vals, LOGT, j, p, ok, cap, &s_ndist[g], &s_full[g]);
        };
        group_products<V, true, G, 2, decltype(get), decltype(sink), true>(Arp[row], Arp[row + 1], gt, s_en[g], Bcol,
                                                                            Bval, get, sink);
    }
    group_sync<WPR>();
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
    if (lane == kWave - 1) s_scan[g][wg] = incl;
    group_sync<WPR>();
    int wbase = 0, total = 0;
    for (int w = 0; w < WPR; ++w) {
        const int t = s_scan[g][w];
        if (w < wg) wbase += t;
        total += t;
    }
    const bool ok = active && !s_full[g] && total <= cap && stage_off[row] + cap <= stage_cap;
    order_row_entries<T, WPR, SPT>(kr, vr, keys, vals, s_scan[g], total, wbase, incl, cnt, ncols, gt);
    if (active) {
        if (ok) {
            const long long o = stage_off[row];
            for (int t = gt; t < total; t += G) {
                scol[o + t] = keys[t];
                sval[o + t] = (V)vals[t];
            }
        }
        if (gt == 0) {
            status[row] = ok ? 1 : 0;
            if (ok) nnzc[row] = total;
        }
    }
    group_sync<WPR>();
    }
}

// Rows completed by the fused pass leave the two-phase plan (one global
// atomic per block for their number and one for their entries).
__global__ __launch_bounds__(256) void k_fused_mark(int m, const unsigned char *__restrict__ fbin,
                                                    const unsigned char *__restrict__ status,
                                                    const int *__restrict__ nnzc, unsigned char *__restrict__ sym_bin,
                                                    int *fused_ok, unsigned long long *fused_entries, const int *err)
{
    // grid-stride over the rows; the block's totals go out with one atomic
    // per counter (a block per 256 rows would serialise thousands of
    // atomics on the two counters)
    if (stopped(err)) return;
    __shared__ int s_ok;
    __shared__ unsigned long long s_ent;
    if (threadIdx.x == 0) {
        s_ok = 0;
        s_ent = 0;
    }
    __syncthreads();
    int ok = 0;
    unsigned long long ent = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        if (fbin[i] != kBinEmpty && status[i] == 1) {
            sym_bin[i] = kBinEmpty;
            ++ok;
            ent += (unsigned long long)nnzc[i];
        }
    }
    ok = wave_sum(ok);
    ent = wave_sum(ent);
    if (lane_id() == 0 && ok) {
        atomicAdd(&s_ok, ok);
        atomicAdd(&s_ent, ent);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_ok) {
        atomicAdd(fused_ok, s_ok);
        atomicAdd(fused_entries, s_ent);
    }
}

// Copies the staged rows of the fused pass to their final offsets in C
// (one wave per row, coalesced, non-temporal stores).
template <typename V>
__global__ __launch_bounds__(256) void k_fused_copy(const int *__restrict__ rows, int nrows,
                                                    const unsigned char *__restrict__ status,
                                                    const long long *__restrict__ stage_off,
                                                    const int *__restrict__ scol, const V *__restrict__ sval,
                                                    const long long *__restrict__ Crp, int *__restrict__ Ccol,
                                                    V *__restrict__ Cval)
{
    const int r = blockIdx.x * 4 + threadIdx.x / kWave;
    if (r >= nrows) return;
    const int row = rows[r];
    if (status[row] != 1) return;
    const long long o = stage_off[row], d = Crp[row];
    const int n = (int)(Crp[row + 1] - d);
    for (int t = lane_id(); t < n; t += kWave) {
        store_c(&Ccol[d + t], scol[o + t]);
        store_c(&Cval[d + t], sval[o + t]);
    }
}

}  // namespace smash
