// Training of the learned bath closure on the GPU.
//
// The closure stands in for the bath force of eq:Pz_update-LB, which is a linear causal filter of
// the polarization history (eq:EOM_LorentzBath-2).  Training data are polarization and field
// trajectories recorded from the explicit Lorentz-Bath solver; the target force along each
// trajectory is recomputed here in FP64 by running the bath recurrence eq:Yzj_finite_difference
// driven by the recorded P (the force that produced each recorded P^{n+3/2}).
//
// Network (width 32, K = 4): x = [E s_E, P s_P, V s_V, h], z1 = act(W1 x + b1),
// z2 = act(W2 z1 + b2), o = W3 z2 + b3; h <- h + o[0:4]; prediction o[4] of the scaled force
// S s_S.  Loss = mean of (o[4] - S s_S)^2.  Truncated backpropagation through time over windows
// of W steps, taken in order from the start of the record: the hidden state entering window c is
// carried from the forward pass of window c - 1 (a constant for the gradient).  One Adam step per
// window (all trajectories at once).
//
// Kernels: bath-force replay (FP64), input moments (FP64 sums) and packing, forward (one thread
// per trajectory, weights uniform and read through the constant address space; activations kept
// for the backward pass), backward (deltas per step), the weight-gradient contraction (LDS-staged
// tiles, FP32 tile sums accumulated in FP64), the block-partial reduction and Adam (FP64 master
// weights, FP32 copy for the passes).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fdtdb.h"
#include "fdtdb_internal.h"

namespace fdtdb {
namespace train {

constexpr int NIN = 7, NK = 4, NOUT = 5, WID = kClosureWidth;
constexpr int NP = kClosureParams;
// activation record per step: x (7), z1 (32), z2 (32)
constexpr int A_X = 0, A_Z1 = 7, A_Z2 = 39, NACT = 71;
// delta record per step: do (5), da2 (32), da1 (32)
constexpr int D_O = 0, D_A2 = 5, D_A1 = 37, NDEL = 69;
// parameter offsets (row major)
constexpr int P_W1 = 0, P_B1 = P_W1 + WID * NIN, P_W2 = P_B1 + WID, P_B2 = P_W2 + WID * WID, P_W3 = P_B2 + WID,
              P_B3 = P_W3 + NOUT * WID;
static_assert(P_B3 + NOUT == NP, "closure layout");
constexpr int TB = 256;          // threads per block
constexpr int TILE = 64;         // samples per weight-gradient tile
constexpr int LDS_STRIDE = TILE + 1;

typedef const __attribute__((address_space(4))) float *cfp;

template <int ACT>
__device__ __forceinline__ float act_f(float a) {
    return ACT == 0 ? tanh_f(a) : a;
}
template <int ACT>
__device__ __forceinline__ float dact_f(float z) {
    return ACT == 0 ? 1.0f - z * z : 1.0f;
}

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[TB / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < TB / 64; ++q) s += red[q];
    return s;
}

// ------------------------------------------------------------------------------- data preparation
// S[t][i] for the recorded P: P_full[0] = 0 (rest), P_full[t + 1] = Prec[t][i].  Modes in groups of
// 8 (the force of each group is added to S).  coef per mode: a_j, b_j, c_j, k_j.
__global__ __launch_bounds__(TB) void k_replay(const float *Prec, long long N, long long T, const double *coef, int j0,
                                               int nj, double dt, double *S) {
    const long long i = blockIdx.x * (long long)TB + threadIdx.x;
    if (i >= N) return;
    double y0[8], y1[8], a[8], b[8], c[8], k[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const bool on = q < nj;
        a[q] = on ? coef[4 * (j0 + q)] : 0.0;
        b[q] = on ? coef[4 * (j0 + q) + 1] : 0.0;
        c[q] = on ? coef[4 * (j0 + q) + 2] : 0.0;
        k[q] = on ? coef[4 * (j0 + q) + 3] : 0.0;
        y0[q] = 0.0;      // Y^{m}
        y1[q] = 0.0;      // Y^{m-1}
    }
    double pm1 = 0.0, p0 = 0.0;   // P^{m-1}, P^{m}
    for (long long t = 0; t < T; ++t) {
        double f = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) f += k[q] * (a[q] * y0[q] + b[q] * y1[q]);
        f *= 0.5 * dt;
        const double pn = (double)Prec[t * N + i];   // P^{m+1}
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double yn = a[q] * y0[q] + (b[q] + 1.0) * y1[q] + c[q] * (pn - pm1);
            y1[q] = y0[q];
            y0[q] = yn;
        }
        pm1 = p0;
        p0 = pn;
        double *d = S + t * N + i;
        *d = (j0 == 0 ? 0.0 : *d) + f;
    }
}

// sums of E^2, P^2, V^2, S^2 over the record (block partials)
__global__ __launch_bounds__(TB) void k_moments(const float *Erec, const float *Prec, const double *S, long long N,
                                                long long T, double inv_dt, double *part) {
    double se = 0.0, sp = 0.0, sv = 0.0, ss = 0.0;
    const long long tot = N * T;
    for (long long q = blockIdx.x * (long long)TB + threadIdx.x; q < tot; q += (long long)gridDim.x * TB) {
        const long long t = q / N;
        const double e = Erec[q];
        const double p = t > 0 ? (double)Prec[q - N] : 0.0;          // P^{m}
        const double pp = t > 1 ? (double)Prec[q - 2 * N] : 0.0;     // P^{m-1}
        const double v = (p - pp) * inv_dt;
        se += e * e;
        sp += p * p;
        sv += v * v;
        ss += S[q] * S[q];
    }
    se = block_sum(se);
    __syncthreads();
    sp = block_sum(sp);
    __syncthreads();
    sv = block_sum(sv);
    __syncthreads();
    ss = block_sum(ss);
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x] = se;
        part[4 * blockIdx.x + 1] = sp;
        part[4 * blockIdx.x + 2] = sv;
        part[4 * blockIdx.x + 3] = ss;
    }
}

// scales = 1 / rms of each input (1 where the rms vanishes)
__global__ void k_scales(const double *part, int nblk, double count, double *scales) {
    if (threadIdx.x >= 4) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[4 * b + threadIdx.x];
    const double rms = sqrt(s / count);
    scales[threadIdx.x] = rms > 0.0 ? 1.0 / rms : 1.0;
}

// X[t][3][N] = (E s_E, P s_P, V s_V), Y[t][N] = S s_S (FP32)
__global__ __launch_bounds__(TB) void k_pack(const float *Erec, const float *Prec, const double *S, long long N,
                                             long long T, double inv_dt, const double *scales, float *X, float *Y) {
    const long long tot = N * T;
    const double sE = scales[0], sP = scales[1], sV = scales[2], sS = scales[3];
    for (long long q = blockIdx.x * (long long)TB + threadIdx.x; q < tot; q += (long long)gridDim.x * TB) {
        const long long t = q / N, i = q - t * N;
        const double p = t > 0 ? (double)Prec[q - N] : 0.0;
        const double pp = t > 1 ? (double)Prec[q - 2 * N] : 0.0;
        float *x = X + t * 3 * N + i;
        x[0] = (float)(Erec[q] * sE);
        x[N] = (float)(p * sP);
        x[2 * N] = (float)((p - pp) * inv_dt * sV);
        Y[q] = (float)(S[q] * sS);
    }
}

// ------------------------------------------------------------------------------- forward / backward
template <int ACT>
__global__ __launch_bounds__(TB) void k_forward(const float *X, const float *Y, const float *wt_, float4 *hcarry,
                                                float *act, float *res, double *lossp, long long N, int W, long long t0) {
    // weights in the transposed layout: one contiguous row per input feature, every output unit an
    // independent accumulator
    const cfp w = (cfp)wt_;
    const long long i = blockIdx.x * (long long)TB + threadIdx.x;
    const bool live = i < N;
    double lsum = 0.0;
    if (live) {
        float4 h = hcarry[i];
        for (int t = 0; t < W; ++t) {
            const float *xs = X + (t0 + t) * 3 * N + i;
            const float x[NIN] = {xs[0], xs[N], xs[2 * N], h.x, h.y, h.z, h.w};
            float *ar = act + (long long)t * NACT * N + i;
#pragma unroll
            for (int v = 0; v < NIN; ++v) ar[(A_X + v) * N] = x[v];
            float z1[WID], z2[WID];
#pragma unroll
            for (int u = 0; u < WID; ++u) z1[u] = w[P_B1 + u];
#pragma unroll
            for (int v = 0; v < NIN; ++v) {
#pragma unroll
                for (int u = 0; u < WID; ++u) z1[u] = fmaf(w[P_W1 + v * WID + u], x[v], z1[u]);
                __asm__ volatile("" ::: "memory");
            }
#pragma unroll
            for (int u = 0; u < WID; ++u) {
                z1[u] = act_f<ACT>(z1[u]);
                ar[(A_Z1 + u) * N] = z1[u];
                z2[u] = w[P_B2 + u];
            }
#pragma unroll
            for (int v = 0; v < WID; ++v) {
#pragma unroll
                for (int u = 0; u < WID; ++u) z2[u] = fmaf(w[P_W2 + v * WID + u], z1[v], z2[u]);
                __asm__ volatile("" ::: "memory");
            }
            float o[NOUT];
#pragma unroll
            for (int k = 0; k < NOUT; ++k) o[k] = w[P_B3 + k];
#pragma unroll
            for (int u = 0; u < WID; ++u) {
                z2[u] = act_f<ACT>(z2[u]);
                ar[(A_Z2 + u) * N] = z2[u];
#pragma unroll
                for (int k = 0; k < NOUT; ++k) o[k] = fmaf(w[P_W3 + u * NOUT + k], z2[u], o[k]);
                if ((u & 3) == 3) __asm__ volatile("" ::: "memory");
            }
            const float r = o[4] - Y[(t0 + t) * N + i];
            res[(long long)t * N + i] = r;
            lsum += (double)r * (double)r;
            h.x += o[0];
            h.y += o[1];
            h.z += o[2];
            h.w += o[3];
        }
        hcarry[i] = h;
    }
    const double s = block_sum(lsum);
    if (threadIdx.x == 0) lossp[blockIdx.x] = s;
}

template <int ACT>
__global__ __launch_bounds__(TB) void k_backward(const float *w_, const float *act, const float *res, float *del,
                                                 long long N, int W, float scale) {
    const cfp w = (cfp)w_;
    const long long i = blockIdx.x * (long long)TB + threadIdx.x;
    if (i >= N) return;
    float dh[NK] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int t = W - 1; t >= 0; --t) {
        const float *ar = act + (long long)t * NACT * N + i;
        float *dr = del + (long long)t * NDEL * N + i;
        const float d_o[NOUT] = {dh[0], dh[1], dh[2], dh[3], scale * res[(long long)t * N + i]};
#pragma unroll
        for (int k = 0; k < NOUT; ++k) dr[(D_O + k) * N] = d_o[k];
        // da2 = (W3^T do) * act'(z2)
        float g[WID];
#pragma unroll
        for (int u = 0; u < WID; ++u) g[u] = 0.0f;
#pragma unroll
        for (int k = 0; k < NOUT; ++k) {
#pragma unroll
            for (int u = 0; u < WID; ++u) g[u] = fmaf(w[P_W3 + k * WID + u], d_o[k], g[u]);
            __asm__ volatile("" ::: "memory");
        }
        float da2[WID];
#pragma unroll
        for (int u = 0; u < WID; ++u) {
            da2[u] = g[u] * dact_f<ACT>(ar[(A_Z2 + u) * N]);
            dr[(D_A2 + u) * N] = da2[u];
        }
        // da1 = (W2^T da2) * act'(z1)
#pragma unroll
        for (int v = 0; v < WID; ++v) g[v] = 0.0f;
#pragma unroll
        for (int u = 0; u < WID; ++u) {
#pragma unroll
            for (int v = 0; v < WID; ++v) g[v] = fmaf(w[P_W2 + u * WID + v], da2[u], g[v]);
            __asm__ volatile("" ::: "memory");
        }
        float da1[WID];
#pragma unroll
        for (int v = 0; v < WID; ++v) {
            da1[v] = g[v] * dact_f<ACT>(ar[(A_Z1 + v) * N]);
            dr[(D_A1 + v) * N] = da1[v];
        }
        // dx = W1^T da1; the hidden-state part flows into the previous step
        float dx[NK] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int u = 0; u < WID; ++u) {
#pragma unroll
            for (int q = 0; q < NK; ++q) dx[q] = fmaf(w[P_W1 + u * NIN + 3 + q], da1[u], dx[q]);
            if ((u & 7) == 7) __asm__ volatile("" ::: "memory");
        }
#pragma unroll
        for (int q = 0; q < NK; ++q) dh[q] += dx[q];
    }
}

// Weight gradients: every parameter block is an outer product of a delta vector and an activation
// vector (+ a constant-1 column for the biases) summed over samples (window steps x trajectories).
// A tile of 64 samples is staged in LDS sample-major (72 floats per sample: activations
// [x0..x6, 1, z1, z2], deltas [do0..4, 0, 0, 0, da2, da1]), and each thread owns a 4 x 4 block of
// one product: per sample one 16-byte read of 4 deltas, one of 4 activations, 16 FMAs.  FP32 sums
// per tile, FP64 across tiles; the two halves of the block take alternate halves of the samples.
constexpr int SROW = 76;           // LDS floats per sample (72 used; 16-byte aligned rows)
constexpr int A_OFF_X = 0, A_OFF_ONE = 7, A_OFF_Z1 = 8, A_OFF_Z2 = 40;
constexpr int D_OFF_O = 0, D_OFF_A2 = 8, D_OFF_A1 = 40;
constexpr int NTASK = 106;         // 4 x 4 tasks: W1|b1 16, W2 64, b2 8, W3 16, b3 2

struct Task {
    int doff, aoff;                // offsets of the 4 deltas / 4 activations in an LDS sample row
    int kind, r0, c0;              // 0: W1|b1, 1: W2, 2: b2, 3: W3, 4: b3; first row / column
};
__device__ __forceinline__ Task task_of(int id) {
    Task k;
    if (id < 16) { k.kind = 0; k.r0 = 4 * (id >> 1); k.c0 = 4 * (id & 1); k.doff = D_OFF_A1 + k.r0; k.aoff = A_OFF_X + k.c0; }
    else if (id < 80) { const int q = id - 16; k.kind = 1; k.r0 = 4 * (q >> 3); k.c0 = 4 * (q & 7); k.doff = D_OFF_A2 + k.r0; k.aoff = A_OFF_Z1 + k.c0; }
    else if (id < 88) { const int q = id - 80; k.kind = 2; k.r0 = 4 * q; k.c0 = 0; k.doff = D_OFF_A2 + k.r0; k.aoff = 4; }
    else if (id < 104) { const int q = id - 88; k.kind = 3; k.r0 = 4 * (q >> 3); k.c0 = 4 * (q & 7); k.doff = D_OFF_O + k.r0; k.aoff = A_OFF_Z2 + k.c0; }
    else { const int q = id - 104; k.kind = 4; k.r0 = 4 * q; k.c0 = 0; k.doff = D_OFF_O + k.r0; k.aoff = 4; }
    return k;
}
// parameter index of (r, c) of a task's 4 x 4 block, or -1 for padding
__device__ __forceinline__ int task_param(const Task &k, int r, int c) {
    const int row = k.r0 + r, col = k.c0 + c;
    switch (k.kind) {
        case 0: return col < 7 ? P_W1 + row * NIN + col : P_B1 + row;          // column 7 is the constant 1
        case 1: return P_W2 + row * WID + col;
        case 2: return c == 3 ? P_B2 + row : -1;                               // activation offset 4 + 3 = the 1
        case 3: return row < NOUT ? P_W3 + row * WID + col : -1;
        default: return (c == 3 && row < NOUT) ? P_B3 + row : -1;
    }
}

// partial[block][e] = sum over this block's tiles of delta * activation
__global__ __launch_bounds__(TB) void k_wgrad(const float *act, const float *del, long long N, int W, int tiles_per_block,
                                              double *partial) {
    __shared__ float sa[TILE * SROW];
    __shared__ float sd[TILE * SROW];
    __shared__ double comb[NTASK][16];
    const long long ntx = (N + TILE - 1) / TILE;
    const long long ntiles = ntx * W;
    const int half = threadIdx.x >> 7, id = threadIdx.x & 127;
    const bool busy = id < NTASK;
    const Task K = task_of(busy ? id : 0);
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    // staging: thread (s = tid mod 64, f0 = tid / 64) moves features f0, f0 + 4, ... of sample s; the next
    // tile's values are loaded into registers while the current tile is being multiplied
    constexpr int NST = (NACT + NDEL) * TILE / TB;
    static_assert((NACT + NDEL) * TILE % TB == 0, "staging split");
    const int s_me = threadIdx.x & (TILE - 1), f0 = threadIdx.x / TILE;
    float pre[NST];
    auto fetch = [&](long long tile) {
        const long long t = tile / ntx, i = (tile - t * ntx) * TILE + s_me;
        const bool ok = i < N;
#pragma unroll
        for (int r = 0; r < NST; ++r) {
            const int f = f0 + r * (TB / TILE);
            const float *src = f < NACT ? act + (t * NACT + f) * N : del + (t * NDEL + (f - NACT)) * N;
            pre[r] = ok ? src[i] : 0.0f;
        }
    };
    const long long first = (long long)blockIdx.x * tiles_per_block;
    const long long last = first + tiles_per_block < ntiles ? first + tiles_per_block : ntiles;
    if (first < last) fetch(first);
    for (long long tile = first; tile < last; ++tile) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NST; ++r) {
            const int f = f0 + r * (TB / TILE);
            if (f < NACT) {
                const int col = f < NIN ? A_OFF_X + f : (f < A_Z2 ? A_OFF_Z1 + (f - A_Z1) : A_OFF_Z2 + (f - A_Z2));
                sa[s_me * SROW + col] = pre[r];
            } else {
                const int g = f - NACT;
                const int col = g < NOUT ? D_OFF_O + g : (g < D_A1 ? D_OFF_A2 + (g - D_A2) : D_OFF_A1 + (g - D_A1));
                sd[s_me * SROW + col] = pre[r];
            }
        }
        if (threadIdx.x < TILE) {
            sa[s_me * SROW + A_OFF_ONE] = 1.0f;
            sd[s_me * SROW + 5] = 0.0f;
            sd[s_me * SROW + 6] = 0.0f;
            sd[s_me * SROW + 7] = 0.0f;
        }
        __syncthreads();
        if (tile + 1 < last) fetch(tile + 1);
        if (busy) {
            float f[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) f[q] = 0.0f;
            for (int s = half; s < TILE; s += 2) {
                const float4 d = *reinterpret_cast<const float4 *>(sd + s * SROW + K.doff);
                const float4 v = *reinterpret_cast<const float4 *>(sa + s * SROW + K.aoff);
                const float dd[4] = {d.x, d.y, d.z, d.w}, vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int c = 0; c < 4; ++c) f[4 * r + c] = fmaf(dd[r], vv[c], f[4 * r + c]);
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] += (double)f[q];
        }
    }
    __syncthreads();
    if (busy && half == 1)
#pragma unroll
        for (int q = 0; q < 16; ++q) comb[id][q] = acc[q];
    __syncthreads();
    if (busy && half == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int e = task_param(K, r, c);
                if (e >= 0) partial[(long long)blockIdx.x * NP + e] = acc[4 * r + c] + comb[id][4 * r + c];
            }
    }
}

// grad[e] = sum_b partial[b][e] (64 entries per block, 4 stripes of partial rows combined in LDS);
// block 0 also adds the window's loss into *lsum (FP64)
__global__ __launch_bounds__(TB) void k_reduce(const double *partial, int nblk, const double *lossp, int nlb,
                                               double loss_scale, double *grad, double *lsum) {
    __shared__ double st[4][64];
    const int e = blockIdx.x * 64 + (threadIdx.x & 63), stripe = threadIdx.x >> 6;
    double s = 0.0;
    if (e < NP)
        for (int b = stripe; b < nblk; b += 4) s += partial[(long long)b * NP + e];
    st[stripe][threadIdx.x & 63] = s;
    __syncthreads();
    if (stripe == 0 && e < NP) grad[e] = st[0][threadIdx.x] + st[1][threadIdx.x] + st[2][threadIdx.x] + st[3][threadIdx.x];
    if (blockIdx.x == 0) {
        __syncthreads();
        double l = 0.0;
        for (int b = threadIdx.x; b < nlb; b += TB) l += lossp[b];
        l = block_sum(l);
        if (threadIdx.x == 0) *lsum += l * loss_scale;
    }
}

// Adam with bias correction (t counts from 1); FP64 master weights, FP32 copy
__global__ __launch_bounds__(TB) void k_adam(double *w64, float *w32, float *wt, double *m, double *v, const double *grad,
                                             double lr, double c1, double c2) {
    const int e = blockIdx.x * TB + threadIdx.x;
    if (e >= NP) return;
    const double g = grad[e];
    if (!(g - g == 0.0)) return;      // a non-finite gradient leaves the parameter alone
    const double mn = 0.9 * m[e] + 0.1 * g;
    const double vn = 0.999 * v[e] + 0.001 * g * g;
    m[e] = mn;
    v[e] = vn;
    const double wn = w64[e] - lr * (mn / c1) / (sqrt(vn / c2) + 1e-8);
    w64[e] = wn;
    w32[e] = (float)wn;
    wt[closure_tpos(e)] = (float)wn;
}

// identity -> tanh: scale so that the tanh network equals the identity network to O(eps^2) in
// its near-linear regime: W1, b1, b2 by eps (pre-activations shrink by eps), W3 by 1 / eps
__global__ __launch_bounds__(TB) void k_embed(double *w64, float *w32, float *wt, double eps) {
    const int e = blockIdx.x * TB + threadIdx.x;
    if (e >= NP) return;
    double f = 1.0;
    if (e < P_W2 || (e >= P_B2 && e < P_W3)) f = eps;
    else if (e >= P_W3 && e < P_B3) f = 1.0 / eps;
    const double wn = w64[e] * f;
    w64[e] = wn;
    w32[e] = (float)wn;
    wt[closure_tpos(e)] = (float)wn;
}

__global__ __launch_bounds__(TB) void k_to_f32(const double *w64, float *w32, float *wt) {
    const int e = blockIdx.x * TB + threadIdx.x;
    if (e < NP) {
        w32[e] = (float)w64[e];
        wt[closure_tpos(e)] = (float)w64[e];
    }
}

__global__ void k_fill4(float4 *p, long long n) {
    const long long i = blockIdx.x * (long long)TB + threadIdx.x;
    if (i < n) p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

__global__ void k_fill(double *p, long long n) {
    const long long i = blockIdx.x * (long long)TB + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace train
}  // namespace fdtdb

using namespace fdtdb;
using namespace fdtdb::train;

// ============================================================================ host runtime
namespace {

thread_local std::string t_err;

fdtdb_status tfail(fdtdb_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return st;
}

#define THIP(x)                                                                                 \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) return tfail(FDTDB_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)
#define TTRY(x)                         \
    do {                                \
        fdtdb_status s_ = (x);          \
        if (s_ != FDTDB_OK) return s_;  \
    } while (0)

unsigned nblk(long long n) { return (unsigned)((n + TB - 1) / TB); }

}  // namespace

struct fdtdb_trainer_s {
    long long N = 0, T = 0;
    int W = 0, act = 0;
    double dt = 0.0;
    int nb = 0;
    hipStream_t stream = nullptr;
    std::vector<void *> allocs;
    double *coef = nullptr;                 // per mode a, b, c, k
    float *Erec = nullptr, *Prec = nullptr; // [T][N]
    double *S = nullptr;                    // [T][N]
    float *X = nullptr, *Y = nullptr;       // [T][3][N], [T][N]
    double *scales = nullptr;               // s_E, s_P, s_V, s_S
    double *mom = nullptr;                  // moment block partials
    int mom_blocks = 1024;
    float *act_buf = nullptr, *del = nullptr, *res = nullptr;
    float4 *h = nullptr;
    double *lossp = nullptr, *partial = nullptr, *grad = nullptr, *lsum = nullptr;
    int wg_blocks = 0, wg_tiles = 0;
    double *w64 = nullptr, *m = nullptr, *v = nullptr;
    double *snap = nullptr;                 // weights, m, v before the current epoch
    float *w32 = nullptr;
    float *wt = nullptr;                    // FP32 weights in the transposed layout (forward pass)
    long long adam_t = 0;
    bool loaded = false, have_w = false;

    DevAllocator mem = current_allocator();
    fdtdb_status alloc(void **p, size_t bytes) {
        if (bytes == 0) bytes = 8;
        hipError_t e = dev_alloc(mem, p, bytes);
        if (e != hipSuccess) return tfail(FDTDB_E_NOMEM, "device allocation of %zu bytes: %s", bytes, hipGetErrorString(e));
        allocs.push_back(*p);
        return FDTDB_OK;
    }
};

namespace {

fdtdb_status zero(fdtdb_trainer_s *t, double *p, long long n) {
    hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(TB), 0, t->stream, p, n);
    THIP(hipGetLastError());
    return FDTDB_OK;
}

// forward + backward + gradient of window c (hidden state taken from t->h)
fdtdb_status window_grad(fdtdb_trainer_s *t, long long c, double loss_scale) {
    const long long N = t->N;
    const int W = t->W;
    const unsigned nb = nblk(N);
    if (t->act == 0)
        hipLaunchKernelGGL(k_forward<0>, dim3(nb), dim3(TB), 0, t->stream, t->X, t->Y, t->wt, t->h, t->act_buf, t->res,
                           t->lossp, N, W, c * W);
    else
        hipLaunchKernelGGL(k_forward<1>, dim3(nb), dim3(TB), 0, t->stream, t->X, t->Y, t->wt, t->h, t->act_buf, t->res,
                           t->lossp, N, W, c * W);
    THIP(hipGetLastError());
    const float scale = (float)(2.0 / ((double)N * W));
    if (t->act == 0)
        hipLaunchKernelGGL(k_backward<0>, dim3(nb), dim3(TB), 0, t->stream, t->w32, t->act_buf, t->res, t->del, N, W, scale);
    else
        hipLaunchKernelGGL(k_backward<1>, dim3(nb), dim3(TB), 0, t->stream, t->w32, t->act_buf, t->res, t->del, N, W, scale);
    THIP(hipGetLastError());
    hipLaunchKernelGGL(k_wgrad, dim3(t->wg_blocks), dim3(TB), 0, t->stream, t->act_buf, t->del, N, W, t->wg_tiles,
                       t->partial);
    THIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce, dim3((NP + 63) / 64), dim3(TB), 0, t->stream, t->partial, t->wg_blocks, t->lossp, (int)nb,
                       loss_scale / ((double)N * W), t->grad, t->lsum);
    THIP(hipGetLastError());
    return FDTDB_OK;
}

}  // namespace

extern "C" {

const char *fdtdb_trainer_last_error(void) { return t_err.c_str(); }

fdtdb_status fdtdb_trainer_create(const fdtdb_trainer_desc *d, fdtdb_trainer *out) {
    if (!d || !out) return tfail(FDTDB_E_INVALID, "null argument");
    *out = nullptr;
    if (d->ntraj < 1 || d->nsteps < 1 || d->window < 1 || d->window > 4096 || d->nsteps % d->window)
        return tfail(FDTDB_E_INVALID, "need ntraj >= 1 and nsteps a multiple of window (1..4096)");
    if (d->activation != 0 && d->activation != 1) return tfail(FDTDB_E_INVALID, "activation must be 0 or 1");
    if (!(d->dt > 0.0)) return tfail(FDTDB_E_INVALID, "dt must be > 0");
    if (d->n_bath < 1 || !d->omega_j || !d->gamma_j || !d->k_j) return tfail(FDTDB_E_INVALID, "need the bath modes");
    auto *t = new fdtdb_trainer_s();
    t->N = d->ntraj;
    t->T = d->nsteps;
    t->W = d->window;
    t->act = d->activation;
    t->dt = d->dt;
    t->nb = d->n_bath;
    t->stream = (hipStream_t)d->hip_stream;
    std::vector<double> coef(4 * (size_t)t->nb);
    for (int j = 0; j < t->nb; j++) {
        const double den = 1.0 + 0.5 * d->gamma_j[j] * d->dt;
        coef[4 * j] = (2.0 - d->omega_j[j] * d->omega_j[j] * d->dt * d->dt) / den;
        coef[4 * j + 1] = -2.0 / den;
        coef[4 * j + 2] = d->k_j[j] * d->dt / (2.0 * den);
        coef[4 * j + 3] = d->k_j[j];
    }
    const long long N = t->N, T = t->T, W = t->W;
    fdtdb_status st = FDTDB_OK;
    auto A = [&](void **p, size_t b) { if (st == FDTDB_OK) st = t->alloc(p, b); };
    A((void **)&t->coef, 8 * coef.size());
    A((void **)&t->Erec, 4 * (size_t)(N * T));
    A((void **)&t->Prec, 4 * (size_t)(N * T));
    A((void **)&t->S, 8 * (size_t)(N * T));
    A((void **)&t->X, 12 * (size_t)(N * T));
    A((void **)&t->Y, 4 * (size_t)(N * T));
    A((void **)&t->scales, 32);
    A((void **)&t->mom, 32 * (size_t)t->mom_blocks);
    A((void **)&t->act_buf, 4 * (size_t)(NACT * W * N));
    A((void **)&t->del, 4 * (size_t)(NDEL * W * N));
    A((void **)&t->res, 4 * (size_t)(W * N));
    A((void **)&t->h, 16 * (size_t)N);
    A((void **)&t->lossp, 8 * (size_t)nblk(N));
    const long long ntiles = ((N + TILE - 1) / TILE) * W;
    t->wg_tiles = (int)std::max<long long>(1, (ntiles + 1023) / 1024);
    t->wg_blocks = (int)((ntiles + t->wg_tiles - 1) / t->wg_tiles);
    A((void **)&t->partial, 8 * (size_t)NP * t->wg_blocks);
    A((void **)&t->grad, 8 * (size_t)NP);
    A((void **)&t->lsum, 8);
    A((void **)&t->w64, 8 * (size_t)NP);
    A((void **)&t->m, 8 * (size_t)NP);
    A((void **)&t->v, 8 * (size_t)NP);
    A((void **)&t->w32, 4 * (size_t)NP);
    A((void **)&t->wt, 4 * (size_t)NP);
    A((void **)&t->snap, 48 * (size_t)NP);
    if (st != FDTDB_OK) { fdtdb_trainer_destroy(t); return st; }
    hipError_t e = hipMemcpy(t->coef, coef.data(), 8 * coef.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) { fdtdb_trainer_destroy(t); return tfail(FDTDB_E_DEVICE, "hipMemcpy: %s", hipGetErrorString(e)); }
    *out = t;
    return FDTDB_OK;
}

fdtdb_status fdtdb_trainer_destroy(fdtdb_trainer t) {
    if (!t) return FDTDB_OK;
    if (t->stream) (void)hipStreamSynchronize(t->stream);
    else (void)hipDeviceSynchronize();
    for (void *p : t->allocs) dev_free(t->mem, p);
    delete t;
    return FDTDB_OK;
}

fdtdb_status fdtdb_trainer_load(fdtdb_trainer t, const float *E, const float *P, int on_device) {
    if (!t || !E || !P) return tfail(FDTDB_E_INVALID, "null argument");
    const long long N = t->N, T = t->T;
    const size_t bytes = 4 * (size_t)(N * T);
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (on_device) THIP(hipDeviceSynchronize());   // the caller's writes to E and P, on any stream, come first
    THIP(hipMemcpyAsync(t->Erec, E, bytes, kind, t->stream));
    THIP(hipMemcpyAsync(t->Prec, P, bytes, kind, t->stream));
    for (int j0 = 0; j0 < t->nb; j0 += 8) {
        hipLaunchKernelGGL(k_replay, dim3(nblk(N)), dim3(TB), 0, t->stream, t->Prec, N, T, t->coef, j0,
                           std::min(8, t->nb - j0), t->dt, t->S);
        THIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_moments, dim3(t->mom_blocks), dim3(TB), 0, t->stream, t->Erec, t->Prec, t->S, N, T,
                       1.0 / t->dt, t->mom);
    THIP(hipGetLastError());
    hipLaunchKernelGGL(k_scales, dim3(1), dim3(64), 0, t->stream, t->mom, t->mom_blocks, (double)(N * T), t->scales);
    THIP(hipGetLastError());
    hipLaunchKernelGGL(k_pack, dim3(2048), dim3(TB), 0, t->stream, t->Erec, t->Prec, t->S, N, T, 1.0 / t->dt,
                       t->scales, t->X, t->Y);
    THIP(hipGetLastError());
    THIP(hipStreamSynchronize(t->stream));
    t->loaded = true;
    return FDTDB_OK;
}

fdtdb_status fdtdb_trainer_get_scales(fdtdb_trainer t, double *scales) {
    if (!t || !scales) return tfail(FDTDB_E_INVALID, "null argument");
    if (!t->loaded) return tfail(FDTDB_E_STATE, "no data loaded");
    THIP(hipMemcpy(scales, t->scales, 32, hipMemcpyDeviceToHost));
    return FDTDB_OK;
}

fdtdb_status fdtdb_trainer_get_targets(fdtdb_trainer t, double *S) {
    if (!t || !S) return tfail(FDTDB_E_INVALID, "null argument");
    if (!t->loaded) return tfail(FDTDB_E_STATE, "no data loaded");
    THIP(hipStreamSynchronize(t->stream));
    THIP(hipMemcpy(S, t->S, 8 * (size_t)(t->N * t->T), hipMemcpyDeviceToHost));
    return FDTDB_OK;
}

fdtdb_status fdtdb_trainer_set_weights(fdtdb_trainer t, const float *w) {
    if (!t || !w) return tfail(FDTDB_E_INVALID, "null argument");
    std::vector<double> w64(NP);
    for (int e = 0; e < NP; e++) {
        if (!std::isfinite(w[e])) return tfail(FDTDB_E_INVALID, "non-finite weight");
        w64[e] = w[e];
    }
    THIP(hipStreamSynchronize(t->stream));
    THIP(hipMemcpy(t->w64, w64.data(), 8 * (size_t)NP, hipMemcpyHostToDevice));
    THIP(hipMemcpy(t->w32, w, 4 * (size_t)NP, hipMemcpyHostToDevice));
    std::vector<float> wt(NP);
    for (int e = 0; e < NP; e++) wt[closure_tpos(e)] = w[e];
    THIP(hipMemcpy(t->wt, wt.data(), 4 * (size_t)NP, hipMemcpyHostToDevice));
    TTRY(zero(t, t->m, NP));
    TTRY(zero(t, t->v, NP));
    THIP(hipStreamSynchronize(t->stream));
    t->adam_t = 0;
    t->have_w = true;
    return FDTDB_OK;
}

fdtdb_status fdtdb_trainer_get_weights(fdtdb_trainer t, float *w) {
    if (!t || !w) return tfail(FDTDB_E_INVALID, "null argument");
    if (!t->have_w) return tfail(FDTDB_E_STATE, "no weights set");
    THIP(hipStreamSynchronize(t->stream));
    THIP(hipMemcpy(w, t->w32, 4 * (size_t)NP, hipMemcpyDeviceToHost));
    return FDTDB_OK;
}

fdtdb_status fdtdb_trainer_set_activation(fdtdb_trainer t, int activation, double eps) {
    if (!t || (activation != 0 && activation != 1)) return tfail(FDTDB_E_INVALID, "bad argument");
    if (activation == 0 && t->act == 1 && t->have_w) {
        if (!(eps > 0.0) || !(eps <= 1.0)) return tfail(FDTDB_E_INVALID, "eps must be in (0, 1]");
        hipLaunchKernelGGL(k_embed, dim3(nblk(NP)), dim3(TB), 0, t->stream, t->w64, t->w32, t->wt, eps);
        THIP(hipGetLastError());
        TTRY(zero(t, t->m, NP));
        TTRY(zero(t, t->v, NP));
        THIP(hipStreamSynchronize(t->stream));
        t->adam_t = 0;
    }
    t->act = activation;
    return FDTDB_OK;
}

fdtdb_status fdtdb_trainer_loss_grad(fdtdb_trainer t, double *loss, double *grad) {
    if (!t || !loss || !grad) return tfail(FDTDB_E_INVALID, "null argument");
    if (!t->loaded || !t->have_w) return tfail(FDTDB_E_STATE, "load data and set weights first");
    const long long nwin = t->T / t->W;
    hipLaunchKernelGGL(k_fill4, dim3(nblk(t->N)), dim3(TB), 0, t->stream, t->h, t->N);
    THIP(hipGetLastError());
    TTRY(zero(t, t->lsum, 1));
    std::vector<double> acc(NP, 0.0), g(NP);
    for (long long c = 0; c < nwin; c++) {
        TTRY(window_grad(t, c, 1.0 / (double)nwin));
        THIP(hipMemcpyAsync(g.data(), t->grad, 8 * (size_t)NP, hipMemcpyDeviceToHost, t->stream));
        THIP(hipStreamSynchronize(t->stream));
        for (int e = 0; e < NP; e++) acc[e] += g[e] / (double)nwin;
    }
    THIP(hipMemcpy(loss, t->lsum, 8, hipMemcpyDeviceToHost));
    for (int e = 0; e < NP; e++) grad[e] = acc[e];
    return FDTDB_OK;
}

fdtdb_status fdtdb_trainer_train(fdtdb_trainer t, int epochs, double lr, double lr_decay, double *loss_per_epoch) {
    if (!t || epochs < 0 || !(lr > 0.0) || !(lr_decay > 0.0)) return tfail(FDTDB_E_INVALID, "bad argument");
    if (!t->loaded || !t->have_w) return tfail(FDTDB_E_STATE, "load data and set weights first");
    const long long nwin = t->T / t->W;
    double rate = lr, best = HUGE_VAL;
    int retries = 0;
    // two snapshots of weights and Adam state: the start of the current epoch and of the one before
    // (the weights an epoch ends with are only judged by the next epoch's loss)
    long long t_snap[2] = {t->adam_t, t->adam_t};
    double rate_snap[2] = {rate, rate};
    int cur = 0;
    for (int ep = 0; ep < epochs;) {
        double *sn = t->snap + 3 * (size_t)NP * cur;
        THIP(hipMemcpyAsync(sn, t->w64, 8 * (size_t)NP, hipMemcpyDeviceToDevice, t->stream));
        THIP(hipMemcpyAsync(sn + NP, t->m, 8 * (size_t)NP, hipMemcpyDeviceToDevice, t->stream));
        THIP(hipMemcpyAsync(sn + 2 * NP, t->v, 8 * (size_t)NP, hipMemcpyDeviceToDevice, t->stream));
        t_snap[cur] = t->adam_t;
        rate_snap[cur] = rate;
        hipLaunchKernelGGL(k_fill4, dim3(nblk(t->N)), dim3(TB), 0, t->stream, t->h, t->N);
        THIP(hipGetLastError());
        TTRY(zero(t, t->lsum, 1));
        for (long long c = 0; c < nwin; c++) {
            TTRY(window_grad(t, c, 1.0 / (double)nwin));
            t->adam_t++;
            const double c1 = 1.0 - std::pow(0.9, (double)t->adam_t), c2 = 1.0 - std::pow(0.999, (double)t->adam_t);
            hipLaunchKernelGGL(k_adam, dim3(nblk(NP)), dim3(TB), 0, t->stream, t->w64, t->w32, t->wt, t->m, t->v, t->grad, rate,
                               c1, c2);
            THIP(hipGetLastError());
        }
        double L = 0.0;
        THIP(hipMemcpyAsync(&L, t->lsum, 8, hipMemcpyDeviceToHost, t->stream));
        THIP(hipStreamSynchronize(t->stream));
        if (!std::isfinite(L) || L > 100.0 * best) {
            // the recurrence ran away: go back to the start of the previous epoch (the first epoch
            // goes back to its own start), halve the rate, and repeat from there
            if (++retries > 12) return tfail(FDTDB_E_DIVERGED, "training diverged (epoch %d)", ep);
            const int back = ep > 0 ? cur ^ 1 : cur;
            const double *sb = t->snap + 3 * (size_t)NP * back;
            THIP(hipMemcpyAsync(t->w64, sb, 8 * (size_t)NP, hipMemcpyDeviceToDevice, t->stream));
            THIP(hipMemcpyAsync(t->m, sb + NP, 8 * (size_t)NP, hipMemcpyDeviceToDevice, t->stream));
            THIP(hipMemcpyAsync(t->v, sb + 2 * NP, 8 * (size_t)NP, hipMemcpyDeviceToDevice, t->stream));
            hipLaunchKernelGGL(k_to_f32, dim3(nblk(NP)), dim3(TB), 0, t->stream, t->w64, t->w32, t->wt);
            THIP(hipGetLastError());
            t->adam_t = t_snap[back];
            rate = 0.5 * rate_snap[back];
            if (ep > 0) ep--;
            cur = back;
            continue;
        }
        best = std::min(best, L);
        if (loss_per_epoch) loss_per_epoch[ep] = L;
        rate *= lr_decay;
        cur ^= 1;
        ep++;
    }
    THIP(hipStreamSynchronize(t->stream));
    return FDTDB_OK;
}

}  // extern "C"
