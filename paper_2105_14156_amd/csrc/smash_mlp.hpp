// smash_mlp.hpp -- the learned row-size predictor: per-row features, MLP
// inference, and the training kernels (forward, backward, Adam).
//
// The network maps six per-row features of C = A * B to log2(1 + nnz(C_i)):
// 6 -> 64 -> 64 -> 1, ReLU hidden layers, FP32, parameters packed as
// W1[64][6], b1[64], W2[64][64], b2[64], w3[64], b3.  A predicted capacity
// per row lets the fused pass size its LDS tables without a symbolic pass.
// Training minimises the mean squared error with Adam (Kingma and Ba 2015)
// on batches of rows whose exact counts come from the symbolic phase.
// Reductions over a batch use fixed orders (no atomics), so training is
// deterministic.  The network is far too small for matrix cores to matter
// (about 4.5K multiply-adds per row); every layer is plain FMA.
#pragma once

#include <hip/hip_runtime.h>

#include "smash_kernels.hpp"

namespace smash {

constexpr int kFeat = 6;
constexpr int kHid = 64;
constexpr int kOW1 = 0;
constexpr int kOB1 = kOW1 + kHid * kFeat;
constexpr int kOW2 = kOB1 + kHid;
constexpr int kOB2 = kOW2 + kHid * kHid;
constexpr int kOW3 = kOB2 + kHid;
constexpr int kOB3 = kOW3 + kHid;
constexpr int kParams = kOB3 + 1;     // 4673

// Features of each row i (one wave per row): log2(1 + x) of nnz(A_i), the
// products ub_i, max_k nnz(B_k), min_k nnz(B_k), min(ub_i, cols) and
// sum_k nnz(B_k)^2 / ub_i.  Also ub_i and max_k nnz(B_k) for the capacity
// clamp (nullable).
__global__ __launch_bounds__(256) void k_features(int m, int ncols, const int *__restrict__ Arp,
                                                  const int *__restrict__ Acol, const int *__restrict__ Brp,
                                                  float *__restrict__ feats, long long *__restrict__ ub_out,
                                                  int *__restrict__ maxb_out)
{
    const int lane = lane_id();
    const int row = blockIdx.x * 4 + threadIdx.x / kWave;
    if (row >= m) return;
    const int e0 = Arp[row], e1 = Arp[row + 1];
    long long ub = 0;
    double sq = 0.0;
    int mx = 0, mn = 0x7fffffff;
    for (int e = e0 + lane; e < e1; e += kWave) {
        const int k = Acol[e];
        const int len = Brp[k + 1] - Brp[k];
        ub += len;
        sq += (double)len * (double)len;
        mx = len > mx ? len : mx;
        mn = len < mn ? len : mn;
    }
    ub = wave_sum(ub);
    sq = wave_sum(sq);
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const int a = __shfl_xor(mx, d, kWave), b = __shfl_xor(mn, d, kWave);
        mx = a > mx ? a : mx;
        mn = b < mn ? b : mn;
    }
    if (lane < kFeat) feats[(long long)row * kFeat + lane] = row_feature(lane, e1 - e0, ub, sq, mx, mn, ncols);
    if (lane == 0) {
        if (ub_out) ub_out[row] = ub;
        if (maxb_out) maxb_out[row] = e1 > e0 ? mx : 0;
    }
}

__device__ __forceinline__ void load_params(float *s_w, const float *__restrict__ theta)
{
    for (int t = threadIdx.x; t < kParams; t += blockDim.x) s_w[t] = theta[t];
}

// Network output for one standardized feature vector; h1/h2 receive the
// hidden activations when non-null.
__device__ __forceinline__ float mlp_eval(const float *s_w, const float x[kFeat], float *h1_out, float *h2_out,
                                          int stride)
{
    float h1[kHid];
#pragma unroll
    for (int i = 0; i < kHid; ++i) {
        float z = s_w[kOB1 + i];
#pragma unroll
        for (int f = 0; f < kFeat; ++f) z = fmaf(s_w[kOW1 + i * kFeat + f], x[f], z);
        h1[i] = z > 0.f ? z : 0.f;
        if (h1_out) h1_out[i * stride] = h1[i];
    }
    float y = s_w[kOB3];
    for (int j = 0; j < kHid; ++j) {
        float z = s_w[kOB2 + j];
#pragma unroll
        for (int i = 0; i < kHid; ++i) z = fmaf(s_w[kOW2 + j * kHid + i], h1[i], z);
        const float h = z > 0.f ? z : 0.f;
        if (h2_out) h2_out[j * stride] = h;
        y = fmaf(s_w[kOW3 + j], h, y);
    }
    return y;
}

// Capacity of a row from the network's output y: clamp(ceil(2^(y + delta)
// - 1), max(maxb, 1), min(ub, cols)), 0 for a row without products.
__device__ __forceinline__ int predicted_capacity(float y, float delta, long long u, int maxb_i, int ncols)
{
    if (u <= 0) return 0;
    const long long hi = u < ncols ? u : ncols;
    const long long lo = maxb_i > 1 ? maxb_i : 1;
    float p = exp2f(y + delta) - 1.f;
    long long c = p < 1.f ? 1 : (p > 2.0e9f ? 2000000000LL : (long long)ceilf(p));
    c = c < lo ? lo : c;
    c = c > hi ? hi : c;
    return (int)c;
}

// A wave whose candidate rows are at most this many evaluates them one at a
// time, a hidden unit per lane, instead of a row per lane.
constexpr int kMlpSparseRows = 8;

// Inference: predicted log2(1 + nnz) and, when cap is given, the capacity
// (predicted_capacity).  With only_above >= 0 the network is evaluated only
// for rows whose exact bound min(ub, cols) exceeds it (the rows a
// prediction can move into the LDS tables); the others get the bound
// itself, and a block without such rows loads no weights.  A wave with many
// candidate rows evaluates a row per lane; a wave with few (where the
// candidates are rare, most lanes of a row-per-lane wave would idle through
// the whole network) takes them one by one with lane j computing hidden
// unit j of both layers, reading the other units' values with v_readlane.
// Both forms add in the same order, so a row's result does not depend on
// which form evaluated it.
__global__ __launch_bounds__(256) void k_mlp_predict(int m, int ncols, const float *__restrict__ feats,
                                                     const float *__restrict__ theta, const float *__restrict__ ms,
                                                     float delta, const long long *__restrict__ ub,
                                                     const int *__restrict__ maxb, float *__restrict__ yhat_out,
                                                     int *__restrict__ cap_out, int only_above)
{
    static_assert(kHid == kWave, "one hidden unit per lane");
    __shared__ float s_w[kParams];
    __shared__ float s_ms[2 * kFeat];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const bool live = i < m;
    const long long ub_i = live && ub ? ub[i] : 0;
    const long long bound = ub_i < ncols ? ub_i : ncols;
    const bool cand = live && (only_above < 0 || bound > only_above);
    if (!__syncthreads_or(cand)) {
        if (live && cap_out) cap_out[i] = (int)bound;
        return;
    }
    load_params(s_w, theta);
    if (threadIdx.x < 2 * kFeat) s_ms[threadIdx.x] = ms[threadIdx.x];
    __syncthreads();
    if (live && !cand && cap_out) cap_out[i] = (int)bound;
    const unsigned long long cm = __builtin_amdgcn_ballot_w64(cand);
    if (__popcll(cm) > kMlpSparseRows) {
        if (!cand) return;
        float x[kFeat];
#pragma unroll
        for (int f = 0; f < kFeat; ++f) x[f] = (feats[(long long)i * kFeat + f] - s_ms[f]) / s_ms[kFeat + f];
        const float y = mlp_eval(s_w, x, nullptr, nullptr, 0);
        if (yhat_out) yhat_out[i] = y;
        if (cap_out) cap_out[i] = predicted_capacity(y, delta, ub[i], maxb[i], ncols);
        return;
    }
    if (!cm) return;
    // few candidates: lane j is hidden unit j; its rows of W1 and W2 are
    // read once from the parameters in global memory (a row of W2 in LDS
    // lies in one bank for every lane)
    float w1[kFeat], w2[kHid];
#pragma unroll
    for (int f = 0; f < kFeat; ++f) w1[f] = theta[kOW1 + lane * kFeat + f];
#pragma unroll
    for (int q = 0; q < kHid; ++q) w2[q] = theta[kOW2 + lane * kHid + q];
    const float b1 = s_w[kOB1 + lane], b2 = s_w[kOB2 + lane];
    const int row0 = i - lane;
    for (unsigned long long mm = cm; mm; mm &= mm - 1) {
        const int l = __ffsll((long long)mm) - 1;
        const int r = row0 + l;
        float x[kFeat];
#pragma unroll
        for (int f = 0; f < kFeat; ++f) x[f] = (feats[(long long)r * kFeat + f] - s_ms[f]) / s_ms[kFeat + f];
        float z = b1;
#pragma unroll
        for (int f = 0; f < kFeat; ++f) z = fmaf(w1[f], x[f], z);
        const float h1 = z > 0.f ? z : 0.f;
        float z2 = b2;
#pragma unroll
        for (int q = 0; q < kHid; ++q)
            z2 = fmaf(w2[q], __int_as_float(__builtin_amdgcn_readlane(__float_as_int(h1), q)), z2);
        const float h2 = z2 > 0.f ? z2 : 0.f;
        float y = s_w[kOB3];
#pragma unroll
        for (int q = 0; q < kHid; ++q)
            y = fmaf(s_w[kOW3 + q], __int_as_float(__builtin_amdgcn_readlane(__float_as_int(h2), q)), y);
        if (lane == l) {
            if (yhat_out) yhat_out[r] = y;
            if (cap_out) cap_out[r] = predicted_capacity(y, delta, ub[r], maxb[r], ncols);
        }
    }
}

// ------------------------------------------------------------ training

// Forward pass of one batch (one thread per sample): hidden activations
// h1, h2 (batch x 64, sample-major), dL/dyhat = 2 (yhat - y) / n, and the
// block's sum of squared errors.
__global__ __launch_bounds__(256) void k_mlp_fwd(int n, const int *__restrict__ idx, const float *__restrict__ feats,
                                                 const float *__restrict__ y, const float *__restrict__ ms,
                                                 const float *__restrict__ theta, float *__restrict__ h1,
                                                 float *__restrict__ h2, float *__restrict__ dy,
                                                 double *__restrict__ sse_part)
{
    __shared__ float s_w[kParams];
    __shared__ float s_ms[2 * kFeat];
    __shared__ double s_tmp[256 / kWave + 1];
    load_params(s_w, theta);
    if (threadIdx.x < 2 * kFeat) s_ms[threadIdx.x] = ms[threadIdx.x];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    double se = 0.0;
    if (s < n) {
        const long long r = idx[s];
        float x[kFeat];
#pragma unroll
        for (int f = 0; f < kFeat; ++f) x[f] = (feats[r * kFeat + f] - s_ms[f]) / s_ms[kFeat + f];
        const float yh = mlp_eval(s_w, x, h1 + (long long)s * kHid, h2 + (long long)s * kHid, 1);
        const float res = yh - y[r];
        dy[s] = 2.f * res / (float)n;
        se = (double)res * (double)res;
    }
    double tot;
    block_excl_scan<double, 256>(se, s_tmp, tot);
    if (threadIdx.x == 0) sse_part[blockIdx.x] = tot;
}

// Output layer gradients: block j < 64 computes dw3[j] = sum_s dy_s h2[s][j]
// and writes dz2[s][j] = dy_s w3[j] [h2[s][j] > 0]; block 64 computes db3.
__global__ __launch_bounds__(256) void k_mlp_grad_out(int n, const float *__restrict__ h2, const float *__restrict__ dy,
                                                      const float *__restrict__ theta, float *__restrict__ dz2,
                                                      float *__restrict__ grad)
{
    __shared__ double s_tmp[256 / kWave + 1];
    const int j = blockIdx.x;
    double acc = 0.0;
    if (j < kHid) {
        const float w = theta[kOW3 + j];
        for (int s = threadIdx.x; s < n; s += 256) {
            const float h = h2[(long long)s * kHid + j];
            acc += (double)dy[s] * (double)h;
            dz2[(long long)s * kHid + j] = h > 0.f ? dy[s] * w : 0.f;
        }
    } else {
        for (int s = threadIdx.x; s < n; s += 256) acc += (double)dy[s];
    }
    double tot;
    block_excl_scan<double, 256>(acc, s_tmp, tot);
    if (threadIdx.x == 0) grad[j < kHid ? kOW3 + j : kOB3] = (float)tot;
}

// Hidden layer 2: block j computes dW2[j][i] = sum_s dz2[s][j] h1[s][i] for
// all i (4 partial sums per i over interleaved samples) and db2[j].
__global__ __launch_bounds__(256) void k_mlp_grad_mid(int n, const float *__restrict__ h1,
                                                      const float *__restrict__ dz2, float *__restrict__ grad)
{
    __shared__ double s_part[4][kHid];
    __shared__ double s_tmp[256 / kWave + 1];
    const int j = blockIdx.x;
    const int i = threadIdx.x % kHid, q = threadIdx.x / kHid;
    double acc = 0.0, accb = 0.0;
    for (int s = q; s < n; s += 4) {
        const float d = dz2[(long long)s * kHid + j];
        acc += (double)d * (double)h1[(long long)s * kHid + i];
        if (i == 0) accb += (double)d;
    }
    s_part[q][i] = acc;
    double totb;
    block_excl_scan<double, 256>(accb, s_tmp, totb);
    if (threadIdx.x < kHid)
        grad[kOW2 + j * kHid + threadIdx.x] =
            (float)(s_part[0][threadIdx.x] + s_part[1][threadIdx.x] + s_part[2][threadIdx.x] + s_part[3][threadIdx.x]);
    if (threadIdx.x == 0) grad[kOB2 + j] = (float)totb;
}

// Back through W2: dz1[s][i] = (sum_j W2[j][i] dz2[s][j]) [h1[s][i] > 0],
// one thread per (sample, i).
__global__ __launch_bounds__(256) void k_mlp_back_h1(int n, const float *__restrict__ h1,
                                                     const float *__restrict__ dz2, const float *__restrict__ theta,
                                                     float *__restrict__ dz1)
{
    __shared__ float s_w2[kHid * kHid];
    for (int t = threadIdx.x; t < kHid * kHid; t += 256) s_w2[t] = theta[kOW2 + t];
    __syncthreads();
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)n * kHid) return;
    const long long s = t / kHid;
    const int i = (int)(t % kHid);
    float acc = 0.f;
    const float *d = dz2 + s * kHid;
#pragma unroll 8
    for (int j = 0; j < kHid; ++j) acc = fmaf(s_w2[j * kHid + i], d[j], acc);
    dz1[t] = h1[t] > 0.f ? acc : 0.f;
}

// Input layer: block i computes dW1[i][f] = sum_s dz1[s][i] x[s][f] and
// db1[i].
__global__ __launch_bounds__(256) void k_mlp_grad_in(int n, const int *__restrict__ idx, const float *__restrict__ feats,
                                                     const float *__restrict__ ms, const float *__restrict__ dz1,
                                                     float *__restrict__ grad)
{
    __shared__ double s_tmp[256 / kWave + 1];
    const int i = blockIdx.x;
    double acc[kFeat + 1] = {0, 0, 0, 0, 0, 0, 0};
    for (int s = threadIdx.x; s < n; s += 256) {
        const float d = dz1[(long long)s * kHid + i];
        const long long r = idx[s];
#pragma unroll
        for (int f = 0; f < kFeat; ++f) acc[f] += (double)d * (double)((feats[r * kFeat + f] - ms[f]) / ms[kFeat + f]);
        acc[kFeat] += (double)d;
    }
    for (int f = 0; f <= kFeat; ++f) {
        double tot;
        block_excl_scan<double, 256>(acc[f], s_tmp, tot);
        if (threadIdx.x == 0) grad[f < kFeat ? kOW1 + i * kFeat + f : kOB1 + i] = (float)tot;
    }
}

// Adam update of every parameter (t counts steps from 1).
__global__ __launch_bounds__(256) void k_adam(int np, float *__restrict__ theta, const float *__restrict__ grad,
                                              float *__restrict__ mom, float *__restrict__ vel, int t, float lr,
                                              float b1, float b2, float eps)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const float g = grad[p];
    const float m = b1 * mom[p] + (1.f - b1) * g;
    const float v = b2 * vel[p] + (1.f - b2) * g * g;
    mom[p] = m;
    vel[p] = v;
    const float mh = m / (1.f - powf(b1, (float)t));
    const float vh = v / (1.f - powf(b2, (float)t));
    theta[p] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace smash
