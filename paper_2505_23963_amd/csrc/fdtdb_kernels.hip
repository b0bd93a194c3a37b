// HIP kernels of the FDTD-Bath time step for gfx950 (MI355X).
//
// One thread owns one cell.  The E kernel of a region reads the cell's E,
// the H values of the curl, the cell's polarization levels and bath modes,
// updates everything in FP64 registers and writes each state word once; the
// H kernel reads E and H and writes H.  The work is HBM-bound (about one flop
// per byte), so there is no matrix-core path: the design goals are single
// pass, coalesced z-fastest streams and 16-byte (4-mode) bath vectors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "fdtdb_internal.h"

namespace fdtdb {

template <typename T>
using vec4_t = typename std::conditional<std::is_same<T, float>::value, float4, double4>::type;

template <typename T>
__device__ __forceinline__ double ldd(const void *p, long long i) {
    return (double)static_cast<const T *>(p)[i];
}

__device__ __forceinline__ double warp_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// block sum of three doubles; result valid in thread 0
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c) {
    __shared__ double red[3][kBlock / 64];
    a = warp_sum(a); b = warp_sum(b); c = warp_sum(c);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) { red[0][w] = a; red[1][w] = b; red[2][w] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = b = c = 0.0;
        for (int q = 0; q < kBlock / 64; ++q) { a += red[0][q]; b += red[1][q]; c += red[2][q]; }
    }
}


// Neighbour at coordinate-1 / coordinate+1 along an axis with the axis boundary rule, without
// branches: the load always reads a valid address (the cell itself when the neighbour lies
// beyond a non-periodic edge) and the value is then selected, so loads stay in one batch.
template <typename T>
__device__ __forceinline__ double at_minus(const void *f, int q, int coord, int stride, int n, int per) {
    const bool in = coord > 0;
    const bool ok = in || per;
    const int id = in ? q - stride : (per ? q + (n - 1) * stride : q);
    const double v = (double)static_cast<const T *>(f)[id];
    return ok ? v : 0.0;
}
// A field one cell below q along z, in a 3D kernel with one cell per thread and threads running
// along z rows: the previous lane's own value when that lane holds cell k - 1 of the row (every lane
// but a row's or a wave's first), else a load with the boundary rule of at_minus
template <typename T>
__device__ __forceinline__ double z_minus_lane(const void *f, T own, int q, int k, int klo, int n, int per) {
    const T sv = __shfl_up(own, 1);
    const bool from_lane = (threadIdx.x & 63) > 0 && k > klo;
    return from_lane ? (double)sv : at_minus<T>(f, q, k, 1, n, per);
}
// The same for a 3D kernel whose waves each cover a 32-cell z chunk of two neighbouring y rows (lanes
// 0-31 row j, lanes 32-63 row j + 1): one cell below along z is the previous lane's within the half,
// one row below along y the lane 32 places back for the upper half; other neighbours are loaded
template <typename T>
__device__ __forceinline__ double minus_lane_pairs(const void *f, T own, int q, int ax, int coord, int stride, int n,
                                                   int per) {
    const int lane = threadIdx.x & 63;
    if (ax == 2) {
        const T sv = __shfl_up(own, 1);
        return (lane & 31) ? (double)sv : at_minus<T>(f, q, coord, stride, n, per);
    }
    if (ax == 1) {
        const T sv = __shfl_up(own, 32);
        return lane >= 32 ? (double)sv : at_minus<T>(f, q, coord, stride, n, per);
    }
    return at_minus<T>(f, q, coord, stride, n, per);
}

// threads of a 3D Lorentz-Bath launch in the two-row wave layout above
__host__ __device__ inline long long pair_threads(const int *ext) {
    return (long long)ext[0] * ((ext[1] + 1) / 2) * ((ext[2] + 31) / 32) * 64;
}
template <typename T>
__device__ __forceinline__ double at_plus(const void *f, int q, int coord, int stride, int n, int per) {
    const bool in = coord < n - 1;
    const bool ok = in || per;
    const int id = in ? q + stride : (per ? q - (n - 1) * stride : q);
    const double v = (double)static_cast<const T *>(f)[id];
    return ok ? v : 0.0;
}

// Bloch-periodic axes (the fields are complex, f(r + n_a e_a) = exp(i phi_a) f(r), held as two real
// grids): a neighbour read that wraps past the lower end returns part p of exp(-i phi_a) (v + i w) and
// one past the upper end part p of exp(+i phi_a) (v + i w), with v this part's value and w the other
// part's; with bs = -sin phi_a on the real part and +sin phi_a on the imaginary part these are
// bc v - bs w and bc v + bs w.  tw == nullptr (a real grid): the plain reads.
template <typename T>
__device__ __forceinline__ double at_minus_bloch(const void *f, const void *tw, int q, int coord, int stride, int n,
                                                 int per, double bc, double bs) {
    const double v = at_minus<T>(f, q, coord, stride, n, per);
    if (tw == nullptr || coord > 0 || !per) return v;
    return bc * v - bs * (double)static_cast<const T *>(tw)[q + (n - 1) * stride];
}
template <typename T>
__device__ __forceinline__ double at_plus_bloch(const void *f, const void *tw, int q, int coord, int stride, int n,
                                                int per, double bc, double bs) {
    const double v = at_plus<T>(f, q, coord, stride, n, per);
    if (tw == nullptr || coord < n - 1 || !per) return v;
    return bc * v + bs * (double)static_cast<const T *>(tw)[q - (n - 1) * stride];
}

typedef const __attribute__((address_space(4))) float *cfptr;

// Thermal bath noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), ten rounds on a 4-word
// counter; each round multiplies words 0 and 2 by fixed constants (high and low halves of the 64-bit
// products), mixes the high halves with words 1 and 3 and the key, and the key advances by two Weyl
// constants between rounds.  Counter (grid cell, step, component, variate / 4), key the material's
// seed: variate v is lane v % 4, mode j takes v = j and P takes v = N_b.
struct Philox4 { unsigned x[4]; };
__device__ __forceinline__ Philox4 philox4x32_10(unsigned c0, unsigned c1, unsigned c2, unsigned c3, unsigned k0,
                                                 unsigned k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        // one 64-bit product per word (a single multiply instruction instead of a high and a low one)
        const unsigned long long p0 = 0xD2511F53ull * c0, p1 = 0xCD9E8D57ull * c2;
        c0 = (unsigned)(p1 >> 32) ^ c1 ^ k0; c1 = (unsigned)p1; c2 = (unsigned)(p0 >> 32) ^ c3 ^ k1; c3 = (unsigned)p0;
    }
    return Philox4{{c0, c1, c2, c3}};
}
// unit-variance variate of a 32-bit word: sqrt(12) (u - 1/2), u = (x + 1/2) / 2^32, computed as
// (x - (2^31 - 1/2)) (sqrt(12) 2^-32): the difference is exact and the constant is sqrt(12) rounded
// to double times a power of two, so the one rounded product is the same value
__device__ __forceinline__ double unit_variate(unsigned x) {
    return ((double)x - 2147483647.5) * (3.4641016151377544 / 4294967296.0);
}

// soft-current term dt J(t_n) profile / eps of component c at cell (i, j, k)
__device__ __forceinline__ double source_term(const EArgs &a, const double *amp, int c, int i, int j, int k) {
    double s = 0.0;
#pragma unroll
    for (int n = 0; n < kMaxSources; ++n) {
        if (n >= a.nsrc) break;
        const SourceArg &S = a.src[n];
        if (S.comp != c) continue;
        if (i < S.lo[0] || i >= S.hi[0] || j < S.lo[1] || j >= S.hi[1] || k < S.lo[2] || k >= S.hi[2]) continue;
        double prof = 1.0;
        if (S.profile) {
            const long long sl = ((long long)(i - S.lo[0]) * (S.hi[1] - S.lo[1]) + (j - S.lo[1])) * (S.hi[2] - S.lo[2]) + (k - S.lo[2]);
            prof = S.profile[sl];
        }
        s += S.coef * amp[n] * prof;
    }
    return s;
}

// J(t_n) of every source slot (unused slots hold zero), requested together
__device__ __forceinline__ void load_amps(const EArgs &a, double *amp) {
#pragma unroll
    for (int n = 0; n < kMaxSources; ++n) amp[n] = a.clock->amp[n];
}

// per-block energy partials of every monitor that samples this step
__device__ __forceinline__ void energy_partials(const EArgs &a, bool live, int i, int j, int k, double ef, double ep,
                                                double eb) {
    for (int e = 0; e < a.nen; ++e) {
        const EnergyDev &M = a.en[e];
        if ((a.clock->step % M.every) != 0) continue;
        const bool in = live && i >= M.lo[0] && i < M.hi[0] && j >= M.lo[1] && j < M.hi[1] && k >= M.lo[2] && k < M.hi[2];
        double f0 = in ? ef : 0.0, f1 = in ? ep : 0.0, f2 = in ? eb : 0.0;
        block_sum3(f0, f1, f2);
        if (threadIdx.x == 0) {
            double *out = M.partial + (a.block_base + blockIdx.x) * 3;
            out[0] = f0; out[1] = f1; out[2] = f2;
        }
        __syncthreads();
    }
}

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8).  Remap so
// that each XCD walks one contiguous run of the region in memory order: the y-1 / x-1 halo
// rows a block reads were then written or read shortly before by the same XCD and sit in
// its L2.  Bijective for any block count.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, l = b >> 3;
    return x * q + (x < r ? x : r) + l;
}

// the region a block of a launch works on: the launch's own box, or (grouped launch) the entry of
// the region table that holds the block; returns the block index within the region
struct RegV {
    int lo[3], ext[3], ext12;
    double inv_eps;
    void *psi[3][2];
};
template <class A>
__device__ __forceinline__ int pick_region(const A &a, double inv_eps, int b, RegV &R) {
    if (a.nrd > 0) {
        int r = -1;
#pragma unroll
        for (int s = 0; s < kMaxGroup; ++s) r += b >= a.rd->block0[s];
        const RegionDesc &D = a.rd->d[r];
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            R.lo[x] = D.lo[x];
            R.ext[x] = D.ext[x];
            R.psi[x][0] = D.psi[x][0];
            R.psi[x][1] = D.psi[x][1];
        }
        R.ext12 = D.ext12;
        R.inv_eps = D.inv_eps;
        return b - a.rd->block0[r];
    }
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        R.lo[x] = a.lo[x];
        R.ext[x] = a.ext[x];
        R.psi[x][0] = a.psi[x][0];
        R.psi[x][1] = a.psi[x][1];
    }
    R.ext12 = a.ext12;
    R.inv_eps = inv_eps;
    return b;
}

// 4-wide native vectors for non-temporal (streaming) loads and stores
typedef float nv4f __attribute__((ext_vector_type(4)));
typedef double nv4d __attribute__((ext_vector_type(4)));
template <typename T>
using nvec4_t = typename std::conditional<std::is_same<T, float>::value, nv4f, nv4d>::type;

template <int DIM>
__device__ __forceinline__ void unflatten(int t, const int *lo, const int *ext, int ext12, int &i, int &j, int &k) {
    if (DIM == 1) {
        i = lo[0] + t; j = 0; k = 0;
    } else if (DIM == 2) {
        int r = t / ext[1];
        i = lo[0] + r; j = lo[1] + (t - r * ext[1]); k = 0;
    } else {
        int r = t / ext[2];
        k = lo[2] + (t - r * ext[2]);
        int r2 = r / ext[1];
        i = lo[0] + r2;
        j = lo[1] + (r - r2 * ext[1]);
    }
}

// ---------------------------------------------------------------------------------------------
// E / material update, generic form: background (vacuum, dielectric, CPML), Drude, and the
// Lorentz-Bath path for baths too large for the load-first kernel.
// ---------------------------------------------------------------------------------------------
// E / polarization update of a Lorentz-Bath material whose bath force comes from the learned
// closure.  Per E component and cell: x = [E s_E, P s_P, V s_V, h] -> tanh(W1 x + b1) ->
// tanh(W2 z1 + b2) -> o = W3 z2 + b3; h += o[0:4]; the bath force term of eq:Pz_update-LB is
// o[4] / s_S.  Layers 1 and 2 run on the matrix cores as FP32 MFMA 16x16x4 over tiles of 16 cells:
// each wave stages its 64 cells' inputs in LDS, reads them back in the B-operand layout (lane l:
// cell l mod 16 of the tile, feature 4 s + l / 16 at step s), holds W1 and W2 as A operands in
// registers, and writes each layer's output back over the tile's rows; layer 3 (5 outputs) runs on
// the vector ALU on each lane's own row with the weights read through the constant address space.  Every lane of a wave takes part (lanes past the end
// of the region compute on a clamped cell and store nothing).
// ---------------------------------------------------------------------------------------------
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int kClRow = 36;

// Each wave of the closure kernel stages through its own LDS rows only, so a wave-level barrier with
// an LDS fence orders its writes and reads (no block-wide barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}    // LDS row stride (floats): 16 rows x 4 groups of B reads hit 64 banks once

template <int DIM, typename T, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_update_e_closure(const EArgs a) {
    __shared__ float lds[kBlock / 64][64 * kClRow];
    const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, jl = lane & 15;
    float *row = lds[tid >> 6];
    const int t0 = xcd_block(blockIdx.x, gridDim.x) * kBlock + tid;
    const int ncell = a.ext[0] * a.ext12;
    const bool live = t0 < ncell;
    const int t = live ? t0 : ncell - 1;
    constexpr int W = kClosureWidth;
    // layer 3 reads the transposed copy (one contiguous row per input feature)
    const cfptr wt = (cfptr)(a.cw + kClosureParams);
    const cfptr W3T = wt + W * 7 + W + W * W + W, b3 = W3T + 5 * W;
    // layer-2 operands of this lane: A = W2 rows 16 h + (lane mod 16), columns 4 s + lane / 16;
    // accumulator start = b2 of units 16 h + 4 (lane / 16) + v
    const float *W1 = a.cw, *b1v = W1 + W * 7;
    const float *W2 = b1v + W;
    const float *b2 = W2 + W * W;
    float wa[2][8], wa1[2][2];
    f4v bias1[2], bias2[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int s = 0; s < 8; ++s) wa[h][s] = W2[(16 * h + jl) * W + 4 * s + g];
#pragma unroll
        for (int s = 0; s < 2; ++s) wa1[h][s] = 4 * s + g < 7 ? W1[(16 * h + jl) * 7 + 4 * s + g] : 0.0f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            bias1[h][v] = b1v[16 * h + 4 * g + v];
            bias2[h][v] = b2[16 * h + 4 * g + v];
        }
    }
    double ef = 0.0, ep = 0.0;
    bool sample = false;
    if (ENERGY) {
        const long long st = a.clock->step;
        for (int e = 0; e < a.nen; ++e) sample |= (st % a.en[e].every) == 0;
    }
    double amp[kMaxSources];
    load_amps(a, amp);
    int i, j, k;
    unflatten<DIM>(t, a.lo, a.ext, a.ext12, i, j, k);
    const int s0 = a.n[1] * a.n[2], s1 = a.n[2];
    const int q = i * s0 + j * s1 + k;
    const int coord[3] = {i, j, k};
    const int stride[3] = {s0, s1, 1};
    const int m = ((i - a.mlo[0]) * a.mext[1] + (j - a.mlo[1])) * a.mext[2] + (k - a.mlo[2]);
    const double sig = a.sigma ? ldd<T>(a.sigma, m) : a.sigma0;
    const double *cf = a.coef;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (!e_active(DIM, c)) continue;
        const int a1 = curl_a1(c), a2 = curl_a2(c);
        double t1 = 0.0, t2 = 0.0;
        if (axis_live(DIM, a1) && h_active(DIM, a2))
            t1 = ldd<T>(a.H[a2], q) - at_minus<T>(a.H[a2], q, coord[a1], stride[a1], a.n[a1], a.per[a1]);
        if (axis_live(DIM, a2) && h_active(DIM, a1))
            t2 = ldd<T>(a.H[a1], q) - at_minus<T>(a.H[a1], q, coord[a2], stride[a2], a.n[a2], a.per[a2]);
        const double curl = t1 - t2;
        const double srcterm = source_term(a, amp, c, i, j, k);
        T *Ec = static_cast<T *>(a.E[c]);
        T *Pc_ = static_cast<T *>(a.Pcur[c]);
        T *Pn_ = static_cast<T *>(a.Pnew[c]);
        const double Eo = (double)Ec[q];
        const double Pc = (double)Pc_[m], Pp = (double)Pn_[m];
        const double En = Eo + a.inv_eps * (a.dt * curl - (Pc - Pp)) - srcterm;
        float4 *hp = static_cast<float4 *>(a.hid[c]) + m;
        float4 hv = *hp;
        const float x[7] = {(float)(En * a.cscale[0]), (float)(Pc * a.cscale[1]),
                            (float)((Pc - Pp) / a.dt * a.cscale[2]), hv.x, hv.y, hv.z, hv.w};
        // x row to LDS (7 inputs and a zero); then per tile of 16 cells: layer 1 (K = 8) and layer 2
        // (K = 32) on the matrix cores, z1 and then z2 written over the tile's rows
        *reinterpret_cast<float4 *>(row + lane * kClRow) = make_float4(x[0], x[1], x[2], x[3]);
        *reinterpret_cast<float4 *>(row + lane * kClRow + 4) = make_float4(x[4], x[5], x[6], 0.0f);
        wave_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float *src = row + (16 * r + jl) * kClRow + g;
            float *dst = row + (16 * r + jl) * kClRow + 4 * g;
            f4v c0 = bias1[0], c1 = bias1[1];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const float bv = src[4 * s];
                c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa1[0][s], bv, c0, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa1[1][s], bv, c1, 0, 0, 0);
            }
            float z1[8] = {c0[0], c0[1], c0[2], c0[3], c1[0], c1[1], c1[2], c1[3]};
            tanh_n<8>(z1);
            wave_sync();      // the tile's x rows are consumed
            *reinterpret_cast<float4 *>(dst) = make_float4(z1[0], z1[1], z1[2], z1[3]);
            *reinterpret_cast<float4 *>(dst + 16) = make_float4(z1[4], z1[5], z1[6], z1[7]);
            wave_sync();
            f4v acc0 = bias2[0], acc1 = bias2[1];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const float bv = src[4 * s];
                acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[0][s], bv, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[1][s], bv, acc1, 0, 0, 0);
            }
            float zz[8] = {acc0[0], acc0[1], acc0[2], acc0[3], acc1[0], acc1[1], acc1[2], acc1[3]};
            tanh_n<8>(zz);
            wave_sync();      // the tile's z1 rows are consumed
            *reinterpret_cast<float4 *>(dst) = make_float4(zz[0], zz[1], zz[2], zz[3]);
            *reinterpret_cast<float4 *>(dst + 16) = make_float4(zz[4], zz[5], zz[6], zz[7]);
        }
        wave_sync();
        // layer 3 (vector ALU) on this lane's own row
        float z2[W];
#pragma unroll
        for (int u = 0; u < W; u += 4) {
            const float4 v4 = *reinterpret_cast<const float4 *>(row + lane * kClRow + u);
            z2[u] = v4.x; z2[u + 1] = v4.y; z2[u + 2] = v4.z; z2[u + 3] = v4.w;
        }
        wave_sync();
        float o[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) o[q] = b3[q];
#pragma unroll
        for (int u = 0; u < W; ++u) {
#pragma unroll
            for (int q = 0; q < 5; ++q) o[q] = fmaf(W3T[u * 5 + q], z2[u], o[q]);
            if ((u & 3) == 3) __asm__ volatile("" ::: "memory");
        }
        const double force = (double)o[4] * a.cscale[3];
        const double Pnew = cf[0] * sig * En - cf[1] * Pc - cf[2] * Pp - force * cf[5];
        if (live) {
            hv.x += o[0];
            hv.y += o[1];
            hv.z += o[2];
            hv.w += o[3];
            *hp = hv;
            Ec[q] = (T)En;
            Pn_[m] = (T)Pnew;
        }
        if (ENERGY && sample) {
            ef += 0.5 / a.inv_eps * Eo * En;
            const double rho = cf[3] / sig;
            const double vv = (Pc - Pp) / a.dt;
            ep += 0.5 * rho * (vv * vv + cf[4] * Pc * Pp);
        }
    }
    if (ENERGY && sample) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (h_active(DIM, c)) {
                const double h = ldd<T>(a.H[c], q);
                ef += 0.5 * h * h;
            }
        energy_partials(a, live, i, j, k, ef, ep, 0.0);
    }
}


// ---------------------------------------------------------------------------------------------
// EXT (K_BATH only): the thermal / anharmonic terms of an extended bath
template <int DIM, typename T, int KIND, int NG, bool PML, bool ENERGY, bool EXT = false>
__global__ __launch_bounds__(kBlock) void k_update_e(const EArgs a) {
    using V4 = vec4_t<T>;
    RegV R;
    const int t = pick_region(a, a.inv_eps, xcd_block(blockIdx.x, gridDim.x), R) * kBlock + threadIdx.x;
    const bool live = t < R.ext[0] * R.ext12;
    double ef = 0.0, ep = 0.0, eb = 0.0;   // energy densities of this cell (when sampled)
    bool sample = false;
    if (ENERGY) {
        const long long st = a.clock->step;
        for (int e = 0; e < a.nen; ++e) sample |= (st % a.en[e].every) == 0;
    }
    int i = 0, j = 0, k = 0;
    if (live) {
        double amp[kMaxSources];
        load_amps(a, amp);
        unflatten<DIM>(t, R.lo, R.ext, R.ext12, i, j, k);
        const int s0 = a.n[1] * a.n[2], s1 = a.n[2];
        const int q = i * s0 + j * s1 + k;
        const int coord[3] = {i, j, k};
        const int stride[3] = {s0, s1, 1};
        int m = 0;
        double sig = a.sigma0;
        if (KIND != K_BACKGROUND) {
            m = ((i - a.mlo[0]) * a.mext[1] + (j - a.mlo[1])) * a.mext[2] + (k - a.mlo[2]);
            if (a.sigma) sig = ldd<T>(a.sigma, m);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (!e_active(DIM, c)) continue;
            const int a1 = curl_a1(c), a2 = curl_a2(c);
            double t1 = 0.0, t2 = 0.0;
            if (axis_live(DIM, a1) && h_active(DIM, a2))
                t1 = ldd<T>(a.H[a2], q) - at_minus_bloch<T>(a.H[a2], a.Htw[a2], q, coord[a1], stride[a1], a.n[a1],
                                                             a.per[a1], a.bcos[a1], a.bsin[a1]);
            if (axis_live(DIM, a2) && h_active(DIM, a1))
                t2 = ldd<T>(a.H[a1], q) - at_minus_bloch<T>(a.H[a1], a.Htw[a1], q, coord[a2], stride[a2], a.n[a2],
                                                             a.per[a2], a.bcos[a2], a.bsin[a2]);
            if (PML) {
                if (R.psi[c][0]) {
                    T *ps = static_cast<T *>(R.psi[c][0]);
                    const double psi = a.pml_b[a1][coord[a1]] * (double)__builtin_nontemporal_load(ps + t) + a.pml_c[a1][coord[a1]] * t1;
                    __builtin_nontemporal_store((T)psi, ps + t);
                    t1 += psi;
                }
                if (R.psi[c][1]) {
                    T *ps = static_cast<T *>(R.psi[c][1]);
                    const double psi = a.pml_b[a2][coord[a2]] * (double)__builtin_nontemporal_load(ps + t) + a.pml_c[a2][coord[a2]] * t2;
                    __builtin_nontemporal_store((T)psi, ps + t);
                    t2 += psi;
                }
            }
            const double curl = t1 - t2;
            const double srcterm = source_term(a, amp, c, i, j, k);
            T *Ec = static_cast<T *>(a.E[c]);
            const double Eo = (double)Ec[q];
            double En;
            if (KIND == K_BACKGROUND) {
                En = Eo + R.inv_eps * (a.dt * curl) - srcterm;
                if (ENERGY && sample) ef += 0.5 / R.inv_eps * Eo * En;
            } else if (KIND == K_DRUDE) {
                T *Vp = static_cast<T *>(a.Pcur[c]);
                const double V = (double)__builtin_nontemporal_load(Vp + m);
                En = Eo + R.inv_eps * (a.dt * curl - V) - srcterm;
                __builtin_nontemporal_store((T)(a.coef[0] * En + a.coef[1] * V), Vp + m);
                if (ENERGY && sample) {
                    ef += 0.5 / R.inv_eps * Eo * En;
                    const double v = V / a.dt;
                    ep += 0.5 * a.coef[2] * v * v;
                }
            } else if (KIND == K_MULTI) {
                // sum of Lorentz / Drude terms: E sees the sum of their increments.  A Lorentz term keeps its two
                // levels (ping-pong) and advances by its three-level update, P' = cE E - cP P - cPm P_prev; a Drude
                // term keeps its increment V = P^{n+1/2} - P^{n-1/2} (no restoring force, so P itself never enters)
                // and advances by V' = cE E + cV V, written to the other buffer (coefficients per term in the table)
                T *Pc_ = static_cast<T *>(a.Pcur[c]);
                T *Pn_ = static_cast<T *>(a.Pnew[c]);
                // every term's levels are loaded before any is used (they stream together), then summed in order
                T pcr[kMaxTerms], ppr[kMaxTerms];
#pragma unroll
                for (int p = 0; p < kMaxTerms; ++p) {
                    if (p >= a.nterm) break;
                    const bool drude = a.coef[kCoefHead + kCoefMode * p + 5] != 0.0;
                    pcr[p] = Pc_[(long long)p * a.mcells + m];
                    ppr[p] = drude ? (T)0 : Pn_[(long long)p * a.mcells + m];
                }
                double pc[kMaxTerms], pp[kMaxTerms], dsum = 0.0;
#pragma unroll
                for (int p = 0; p < kMaxTerms; ++p) {
                    if (p >= a.nterm) break;
                    pc[p] = (double)pcr[p];
                    pp[p] = (double)ppr[p];
                    dsum += pc[p] - pp[p];
                }
                En = Eo + R.inv_eps * (a.dt * curl - dsum) - srcterm;
#pragma unroll
                for (int p = 0; p < kMaxTerms; ++p) {
                    if (p >= a.nterm) break;
                    const double *t = a.coef + kCoefHead + kCoefMode * p;
                    const bool drude = t[5] != 0.0;
                    Pn_[(long long)p * a.mcells + m] =
                        (T)(drude ? t[0] * En + t[1] * pc[p] : t[0] * t[6] * En - t[1] * pc[p] - t[2] * pp[p]);
                    if (ENERGY && sample) {
                        const double v = (pc[p] - pp[p]) / a.dt;
                        ep += 0.5 * t[3] * (v * v + t[4] * pc[p] * pp[p]);
                    }
                }
                if (ENERGY && sample) ef += 0.5 / R.inv_eps * Eo * En;
            } else {  // K_BATH (NG == 0: plain Lorentz)
                T *Pc_ = static_cast<T *>(a.Pcur[c]);
                T *Pn_ = static_cast<T *>(a.Pnew[c]);
                const double Pc = (double)Pc_[m], Pp = (double)Pn_[m];
                En = Eo + R.inv_eps * (a.dt * curl - (Pc - Pp)) - srcterm;
                const double *cf = a.coef;
                double S = 0.0;
                V4 yc[NG > 0 ? NG : 1], yp[NG > 0 ? NG : 1];
                const V4 *Yc = static_cast<const V4 *>(a.Ycur[c]);
                V4 *Yn = static_cast<V4 *>(a.Ynew[c]);
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    yc[g] = Yc[(long long)g * a.mcells + m];
                    yp[g] = Yn[(long long)g * a.mcells + m];
                    const double *md = cf + kCoefHead + 4 * g * kCoefMode;
                    S += md[0 * kCoefMode + 3] * (double)yc[g].x + md[0 * kCoefMode + 4] * (double)yp[g].x;
                    S += md[1 * kCoefMode + 3] * (double)yc[g].y + md[1 * kCoefMode + 4] * (double)yp[g].y;
                    S += md[2 * kCoefMode + 3] * (double)yc[g].z + md[2 * kCoefMode + 4] * (double)yp[g].z;
                    S += md[3 * kCoefMode + 3] * (double)yc[g].w + md[3 * kCoefMode + 4] * (double)yp[g].w;
                }
                // thermal / anharmonic bath: each mode's extra term f_j (Langevin force and quartic force,
                // times dt^2 / den_j) enters its own update and, through the substituted Y_j^{n+1}, the
                // P update with the share (dt/2) k_j / A; P's own Langevin force is added to P.  The terms of
                // a group are computed where used (twice: for P, then for Y), not held for all modes.
                constexpr bool ext = NG > 0 && EXT;
                const double *xt = cf + kCoefHead + 4 * NG * kCoefMode;
                const double r = (a.bext & 1) ? sqrt(sig) : 0.0;
                const unsigned step = ext ? (unsigned)a.clock->step : 0u;
                auto ext_terms = [&](int g, double *f) {
                    Philox4 w{};
                    if (a.bext & 1) w = philox4x32_10((unsigned)q, step, (unsigned)c, (unsigned)g, a.key0, a.key1);
                    const double yv[4] = {(double)yc[g].x, (double)yc[g].y, (double)yc[g].z, (double)yc[g].w};
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const double *x = xt + (4 * g + u) * kCoefExt;
                        f[u] = (a.bext & 1) ? x[0] * r * unit_variate(w.x[u]) : 0.0;
                        if (a.bext & 2) f[u] -= x[1] * yv[u] * yv[u] * yv[u];
                    }
                };
                double Pnew = cf[0] * sig * En - cf[1] * Pc - cf[2] * Pp - S;
                if constexpr (ext) {
                    double fs = 0.0;
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        double f[4];
                        ext_terms(g, f);
#pragma unroll
                        for (int u = 0; u < 4; ++u) fs += xt[(4 * g + u) * kCoefExt + 2] * f[u];
                    }
                    Pnew -= fs;
                    if ((a.bext & 1) && cf[6] != 0.0) {      // P's own force (none without gamma0)
                        const int v = a.nb;
                        const Philox4 w = philox4x32_10((unsigned)q, step, (unsigned)c, (unsigned)(v >> 2), a.key0, a.key1);
                        Pnew += cf[6] * r * unit_variate(w.x[v & 3]);
                    }
                }
                Pn_[m] = (T)Pnew;
                const double dP = Pnew - Pp;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const double *md = cf + kCoefHead + 4 * g * kCoefMode;
                    double y[4] = {md[0 * kCoefMode + 0] * (double)yc[g].x + md[0 * kCoefMode + 1] * (double)yp[g].x + md[0 * kCoefMode + 2] * dP,
                                   md[1 * kCoefMode + 0] * (double)yc[g].y + md[1 * kCoefMode + 1] * (double)yp[g].y + md[1 * kCoefMode + 2] * dP,
                                   md[2 * kCoefMode + 0] * (double)yc[g].z + md[2 * kCoefMode + 1] * (double)yp[g].z + md[2 * kCoefMode + 2] * dP,
                                   md[3 * kCoefMode + 0] * (double)yc[g].w + md[3 * kCoefMode + 1] * (double)yp[g].w + md[3 * kCoefMode + 2] * dP};
                    if constexpr (ext) {
                        double f[4];
                        ext_terms(g, f);
#pragma unroll
                        for (int u = 0; u < 4; ++u) y[u] += f[u];
                    }
                    V4 o;
                    o.x = (T)y[0]; o.y = (T)y[1]; o.z = (T)y[2]; o.w = (T)y[3];
                    Yn[(long long)g * a.mcells + m] = o;
                }
                if (ENERGY && sample) {
                    ef += 0.5 / R.inv_eps * Eo * En;
                    const double rho = cf[3] / sig;
                    const double v = (Pc - Pp) / a.dt;
                    ep += 0.5 * rho * (v * v + cf[4] * Pc * Pp);
                    double bsum = 0.0;
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        const double *md = cf + kCoefHead + 4 * g * kCoefMode;
                        const double y0[4] = {(double)yc[g].x, (double)yc[g].y, (double)yc[g].z, (double)yc[g].w};
                        const double y1[4] = {(double)yp[g].x, (double)yp[g].y, (double)yp[g].z, (double)yp[g].w};
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            bsum += (y0[u] - y1[u]) * (y0[u] - y1[u]) / (a.dt * a.dt) + md[u * kCoefMode + 5] * y0[u] * y1[u];
                    }
                    eb += 0.5 * rho * bsum;
                }
            }
            Ec[q] = (T)En;
        }
        if (ENERGY && sample) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (h_active(DIM, c)) {
                    const double h = ldd<T>(a.H[c], q);
                    ef += 0.5 * h * h;
                }
        }
    }
    if (ENERGY && sample) energy_partials(a, live, i, j, k, ef, ep, eb);
}

// ---------------------------------------------------------------------------------------------
// Lorentz-Bath E update, load-first form.  Every load of the cell (E, the H values of the
// curls, both polarization levels, both bath levels of every component) is issued before any
// arithmetic or store, with neighbour reads branch-free, so a wave keeps its whole working set
// in flight; the bath coefficients arrive by value in the kernel arguments (scalar loads).
// E, P and the bath are then advanced in FP64 registers and written once.  Used when the bath
// of all components fits the register budget (components x groups <= 16).  In 2D it also takes
// the wrap rows of a Bloch pair, whose wrapped lower neighbour mixes in the other part (a launch
// elsewhere has no other part and reads as on a real grid).
// ---------------------------------------------------------------------------------------------
template <int DIM, typename T, int NG, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_update_e_bath(const EArgs a, const BathCoef<NG> cf) {
    using V4 = nvec4_t<T>;
    constexpr int NC = DIM == 3 ? 3 : 1;
    // block order: with few bath streams (components x groups <= 6) blocks go in launch order, every
    // XCD streaming next to the others; with more, each XCD takes a contiguous eighth of the layer.
    // Measured per launch: 3D N_b = 8 (3 x 2 groups) 1.69 ms in launch order against 1.73 ms with one
    // row per wave, 1.65 against 1.76 ms with the two-row waves below; 2D N_b = 64 (1 x 16) 0.191
    // against 0.156 ms; 3D N_b = 16 (3 x 4) equal within noise.
    constexpr bool kLaunchOrder = NC * NG <= 6;
    const int t = (kLaunchOrder ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x)) * kBlock + threadIdx.x;
    // 3D without energy sampling: each wave takes a 32-cell z chunk of two neighbouring y rows, so
    // that the y - 1 and z - 1 neighbours of H mostly come from other lanes (measured 1.3 % faster
    // than 64 cells of one row per wave for N_b = 8; 16-cell chunks of four rows were 1.6 % slower)
    constexpr bool kPairs = DIM == 3 && !ENERGY;
    int pi = 0, pj = 0, pk = 0;
    bool live;
    if (kPairs) {
        const int nch = (a.ext[2] + 31) >> 5, ny2 = (a.ext[1] + 1) >> 1;
        const int w = t >> 6, lane = t & 63;
        const int chunk = w % nch, pr = w / nch;
        pi = pr / ny2;
        pj = 2 * (pr - pi * ny2) + (lane >> 5);
        pk = 32 * chunk + (lane & 31);
        live = pi < a.ext[0] && pj < a.ext[1] && pk < a.ext[2];
    } else {
        live = t < a.ext[0] * a.ext12;
    }
    double ef = 0.0, ep = 0.0, eb = 0.0;
    bool sample = false;
    if (ENERGY) {
        const long long st = a.clock->step;
        for (int e = 0; e < a.nen; ++e) sample |= (st % a.en[e].every) == 0;
    }
    int i = 0, j = 0, k = 0;
    if (live) {
        if (kPairs) {
            i = a.lo[0] + pi;
            j = a.lo[1] + pj;
            k = a.lo[2] + pk;
        } else {
            unflatten<DIM>(t, a.lo, a.ext, a.ext12, i, j, k);
        }
        const int s0 = a.n[1] * a.n[2], s1 = a.n[2];
        const int q = i * s0 + j * s1 + k;
        const int coord[3] = {i, j, k};
        const int stride[3] = {s0, s1, 1};
        const int m = ((i - a.mlo[0]) * a.mext[1] + (j - a.mlo[1])) * a.mext[2] + (k - a.mlo[2]);
        const int mcells = (int)a.mcells;
        // ---- phase 1: every load of the cell
        double Eo[NC], Pc[NC], Pp[NC], t1[NC], t2[NC];
        V4 yc[NC][NG], yp[NC][NG];
        // per-cell sigma without a branch: with no sigma array the load reads the cell's own E
        const bool has_sig = a.sigma != nullptr;
        const T *sp = has_sig ? static_cast<const T *>(a.sigma) + m : static_cast<const T *>(a.E[DIM == 3 ? 0 : 2]) + q;
        const T sig_raw = *sp;
#pragma unroll
        for (int ci = 0; ci < NC; ++ci) {
            const int c = DIM == 3 ? ci : 2;
            const int a1 = curl_a1(c), a2 = curl_a2(c);
            t1[ci] = 0.0;
            t2[ci] = 0.0;
            // in 3D neighbours below along z (and, in the two-row layout, along y) come from other lanes
            if (axis_live(DIM, a1) && h_active(DIM, a2)) {
                const T own = static_cast<const T *>(a.H[a2])[q];
                t1[ci] = (double)own -
                         (kPairs ? minus_lane_pairs<T>(a.H[a2], own, q, a1, coord[a1], stride[a1], a.n[a1], a.per[a1])
                          : DIM == 3 && a1 == 2 ? z_minus_lane<T>(a.H[a2], own, q, k, a.lo[2], a.n[2], a.per[2])
                                                : at_minus_bloch<T>(a.H[a2], a.Htw[a2], q, coord[a1], stride[a1], a.n[a1],
                                                                    a.per[a1], a.bcos[a1], a.bsin[a1]));
            }
            if (axis_live(DIM, a2) && h_active(DIM, a1)) {
                const T own = static_cast<const T *>(a.H[a1])[q];
                t2[ci] = (double)own -
                         (kPairs ? minus_lane_pairs<T>(a.H[a1], own, q, a2, coord[a2], stride[a2], a.n[a2], a.per[a2])
                          : DIM == 3 && a2 == 2 ? z_minus_lane<T>(a.H[a1], own, q, k, a.lo[2], a.n[2], a.per[2])
                                                : at_minus_bloch<T>(a.H[a1], a.Htw[a1], q, coord[a2], stride[a2], a.n[a2],
                                                                    a.per[a2], a.bcos[a2], a.bsin[a2]));
            }
            Eo[ci] = (double)static_cast<const T *>(a.E[c])[q];
            // polarization and bath levels are read once and written once per step: stream them
            Pc[ci] = (double)__builtin_nontemporal_load(static_cast<const T *>(a.Pcur[c]) + m);
            Pp[ci] = (double)__builtin_nontemporal_load(static_cast<const T *>(a.Pnew[c]) + m);
            const V4 *Yc = static_cast<const V4 *>(a.Ycur[c]);
            const V4 *Yp = static_cast<const V4 *>(a.Ynew[c]);
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                yc[ci][g] = __builtin_nontemporal_load(Yc + (long long)g * mcells + m);
                yp[ci][g] = __builtin_nontemporal_load(Yp + (long long)g * mcells + m);
            }
        }
        double amp[kMaxSources];
        load_amps(a, amp);
        const double sig = has_sig ? (double)sig_raw : a.sigma0;
        // coefficients: by value for few mode groups; for more (components x groups > 6) from the material's
        // table through the constant address space, the pointer made opaque before each group so that they are
        // re-read through the scalar cache where used rather than held (2D N_b = 64 patch 0.140 against 0.155
        // ms per launch; 3D N_b = 8 0.7 % slower that way, so it keeps the by-value form)
        constexpr bool kTab = NC * NG > 6;
        typedef const __attribute__((address_space(4))) double *cdp;
        cdp co = (cdp)a.coef, md = co;
        auto cm = [&](int g, int u, int q) -> double {
            if constexpr (kTab) return md[u * kCoefMode + q];
            else return cf.md[4 * g + u][q];
        };
        auto group = [&](int g) {
            if constexpr (kTab) {
                asm volatile("" : "+s"(co));
                md = co + kCoefHead + 4 * g * kCoefMode;
            }
        };
        // ---- phase 2: arithmetic and stores
#pragma unroll
        for (int ci = 0; ci < NC; ++ci) {
            const int c = DIM == 3 ? ci : 2;
            const double srcterm = source_term(a, amp, c, i, j, k);
            const double En = Eo[ci] + a.inv_eps * (a.dt * (t1[ci] - t2[ci]) - (Pc[ci] - Pp[ci])) - srcterm;
            double S = 0.0;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                group(g);
                const double yv0[4] = {(double)yc[ci][g].x, (double)yc[ci][g].y, (double)yc[ci][g].z, (double)yc[ci][g].w};
                const double yv1[4] = {(double)yp[ci][g].x, (double)yp[ci][g].y, (double)yp[ci][g].z, (double)yp[ci][g].w};
#pragma unroll
                for (int u = 0; u < 4; ++u) S += cm(g, u, 3) * yv0[u] + cm(g, u, 4) * yv1[u];
            }
            const double Pnew = cf.head[0] * sig * En - cf.head[1] * Pc[ci] - cf.head[2] * Pp[ci] - S;
            const double dP = Pnew - Pp[ci];
            static_cast<T *>(a.E[c])[q] = (T)En;
            __builtin_nontemporal_store((T)Pnew, static_cast<T *>(a.Pnew[c]) + m);
            V4 *Yn = static_cast<V4 *>(a.Ynew[c]);
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                group(g);
                const double yv0[4] = {(double)yc[ci][g].x, (double)yc[ci][g].y, (double)yc[ci][g].z, (double)yc[ci][g].w};
                const double yv1[4] = {(double)yp[ci][g].x, (double)yp[ci][g].y, (double)yp[ci][g].z, (double)yp[ci][g].w};
                double r[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) r[u] = cm(g, u, 0) * yv0[u] + cm(g, u, 1) * yv1[u] + cm(g, u, 2) * dP;
                V4 o;
                o.x = (T)r[0]; o.y = (T)r[1]; o.z = (T)r[2]; o.w = (T)r[3];
                __builtin_nontemporal_store(o, Yn + (long long)g * mcells + m);
            }
            if (ENERGY && sample) {
                ef += 0.5 / a.inv_eps * Eo[ci] * En;
                const double *tab = a.coef;   // energy constants from the global table
                const double rho = tab[3] / sig;
                const double v = (Pc[ci] - Pp[ci]) / a.dt;
                ep += 0.5 * rho * (v * v + tab[4] * Pc[ci] * Pp[ci]);
                double bsum = 0.0;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const double y0[4] = {(double)yc[ci][g].x, (double)yc[ci][g].y, (double)yc[ci][g].z, (double)yc[ci][g].w};
                    const double y1[4] = {(double)yp[ci][g].x, (double)yp[ci][g].y, (double)yp[ci][g].z, (double)yp[ci][g].w};
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        bsum += (y0[u] - y1[u]) * (y0[u] - y1[u]) / (a.dt * a.dt) +
                                tab[kCoefHead + (4 * g + u) * kCoefMode + 5] * y0[u] * y1[u];
                }
                eb += 0.5 * rho * bsum;
            }
        }
        if (ENERGY && sample) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (h_active(DIM, c)) {
                    const double h = ldd<T>(a.H[c], q);
                    ef += 0.5 * h * h;
                }
        }
    }
    if (ENERGY && sample) energy_partials(a, live, i, j, k, ef, ep, eb);
}

// ---------------------------------------------------------------------------------------------
// Lorentz-Bath E update, one (component, cell) per thread: the same arithmetic as the load-first
// kernel above, for 3D baths whose three components' levels do not fit one thread's registers at
// a useful occupancy (components x groups > 6).  Blocks are component-major, so the waves of a
// block stream one component's arrays.  The bath coefficients are read from the material's FP64
// table through the constant address space, the pointer made opaque before each mode group so that
// they are re-read through the scalar cache where used (by value they overflow the scalar registers
// and are read back lane by lane): 512^3 bath launch 6.00 against 6.13 ms.
// ---------------------------------------------------------------------------------------------
// EXT: thermal / anharmonic bath (the extra term f_j of each mode and P's Langevin force, as in the
// general kernel; noise counter (cell, step, component, group))
template <typename T, int NG, int C, bool EXT>
__device__ __forceinline__ void bath_component(const EArgs &a, const BathCoef<NG> &cf, int t) {
    using V4 = nvec4_t<T>;
    int i, j, k;
    unflatten<3>(t, a.lo, a.ext, a.ext12, i, j, k);
    const int s0 = a.n[1] * a.n[2], s1 = a.n[2];
    const int q = i * s0 + j * s1 + k;
    const int coord[3] = {i, j, k};
    const int stride[3] = {s0, s1, 1};
    const int m = ((i - a.mlo[0]) * a.mext[1] + (j - a.mlo[1])) * a.mext[2] + (k - a.mlo[2]);
    const int mcells = (int)a.mcells;
    constexpr int a1 = curl_a1(C), a2 = curl_a2(C);
    const bool has_sig = a.sigma != nullptr;
    const T *sp = has_sig ? static_cast<const T *>(a.sigma) + m : static_cast<const T *>(a.E[C]) + q;
    const T sig_raw = *sp;
    const double t1 = ldd<T>(a.H[a2], q) - at_minus<T>(a.H[a2], q, coord[a1], stride[a1], a.n[a1], a.per[a1]);
    const double t2 = ldd<T>(a.H[a1], q) - at_minus<T>(a.H[a1], q, coord[a2], stride[a2], a.n[a2], a.per[a2]);
    const double Eo = (double)static_cast<const T *>(a.E[C])[q];
    const double Pc = (double)__builtin_nontemporal_load(static_cast<const T *>(a.Pcur[C]) + m);
    const double Pp = (double)__builtin_nontemporal_load(static_cast<const T *>(a.Pnew[C]) + m);
    const V4 *Yc = static_cast<const V4 *>(a.Ycur[C]);
    V4 *Yn = static_cast<V4 *>(a.Ynew[C]);
    V4 yc[NG], yp[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        yc[g] = __builtin_nontemporal_load(Yc + (long long)g * mcells + m);
        yp[g] = __builtin_nontemporal_load(Yn + (long long)g * mcells + m);
    }
    double amp[kMaxSources];
    load_amps(a, amp);
    const double sig = has_sig ? (double)sig_raw : a.sigma0;
    const double En = Eo + a.inv_eps * (a.dt * (t1 - t2) - (Pc - Pp)) - source_term(a, amp, C, i, j, k);
    typedef const __attribute__((address_space(4))) double *cdp;
    cdp co = (cdp)a.coef;
    double S = 0.0;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        asm volatile("" : "+s"(co));
        const cdp md = co + kCoefHead + 4 * g * kCoefMode;
#pragma unroll
        for (int u = 0; u < 4; ++u) S += md[u * kCoefMode + 3] * (double)yc[g][u] + md[u * kCoefMode + 4] * (double)yp[g][u];
    }
    asm volatile("" : "+s"(co));
    double Pnew = co[0] * sig * En - co[1] * Pc - co[2] * Pp - S;
    double fx[EXT ? 4 * NG : 1];
    if constexpr (EXT) {
        const double r = (a.bext & 1) ? sqrt(sig) : 0.0;
        const unsigned step = (unsigned)a.clock->step;
        double fs = 0.0;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            Philox4 w{};
            if (a.bext & 1) w = philox4x32_10((unsigned)q, step, (unsigned)C, (unsigned)g, a.key0, a.key1);
            asm volatile("" : "+s"(co));
            const cdp xt = co + kCoefHead + 4 * NG * kCoefMode + 4 * g * kCoefExt;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double y = (double)yc[g][u];
                double f = 0.0;
                if (a.bext & 1) f = xt[u * kCoefExt + 0] * r * unit_variate(w.x[u]);
                if (a.bext & 2) f -= xt[u * kCoefExt + 1] * y * y * y;
                fx[4 * g + u] = f;
                fs += xt[u * kCoefExt + 2] * f;
            }
        }
        Pnew -= fs;
        asm volatile("" : "+s"(co));
        if ((a.bext & 1) && co[6] != 0.0) {      // P's own force (none without gamma0)
            const int v = a.nb;
            const Philox4 w = philox4x32_10((unsigned)q, step, (unsigned)C, (unsigned)(v >> 2), a.key0, a.key1);
            Pnew += co[6] * r * unit_variate(w.x[v & 3]);
        }
    }
    const double dP = Pnew - Pp;
    static_cast<T *>(a.E[C])[q] = (T)En;
    __builtin_nontemporal_store((T)Pnew, static_cast<T *>(a.Pnew[C]) + m);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        asm volatile("" : "+s"(co));
        const cdp md = co + kCoefHead + 4 * g * kCoefMode;
        V4 o;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double v = md[u * kCoefMode + 0] * (double)yc[g][u] + md[u * kCoefMode + 1] * (double)yp[g][u] + md[u * kCoefMode + 2] * dP;
            if constexpr (EXT) v += fx[4 * g + u];
            o[u] = (T)v;
        }
        __builtin_nontemporal_store(o, Yn + (long long)g * mcells + m);
    }
}

template <typename T, int NG, bool EXT>
__global__ __launch_bounds__(kBathBlock) void k_update_e_bath_c(const EArgs a, const BathCoef<NG> cf) {
    // blocks in launch order within a component (every XCD streaming next to the others): on the 512^3
    // layer 6.30 ms against 6.33 ms with a contiguous share of the component per XCD
    const int nbc = gridDim.x / 3;                  // blocks per component
    const int c = blockIdx.x / nbc;
    const int t = (blockIdx.x - c * nbc) * kBathBlock + threadIdx.x;
    if (t >= a.ext[0] * a.ext12) return;
    if (c == 0) bath_component<T, NG, 0, EXT>(a, cf, t);
    else if (c == 1) bath_component<T, NG, 1, EXT>(a, cf, t);
    else bath_component<T, NG, 2, EXT>(a, cf, t);
}

// ---------------------------------------------------------------------------------------------
// Sum of Lorentz and Drude terms (Sec. II.A) in 3D, one (component, cell) per thread as for the bath:
// E sees the sum of the terms' increments, a Lorentz term advances by its three-level update and a Drude
// term by its increment's (coefficients per term in the table; the same arithmetic, in the same order,
// as the general kernel).  Real grids without CPML terms or energy sampling.
// ---------------------------------------------------------------------------------------------
template <typename T, int C>
__device__ __forceinline__ void multi_component(const EArgs &a, int t) {
    int i, j, k;
    unflatten<3>(t, a.lo, a.ext, a.ext12, i, j, k);
    const int s0 = a.n[1] * a.n[2], s1 = a.n[2];
    const int q = i * s0 + j * s1 + k;
    const int coord[3] = {i, j, k};
    const int stride[3] = {s0, s1, 1};
    const int m = ((i - a.mlo[0]) * a.mext[1] + (j - a.mlo[1])) * a.mext[2] + (k - a.mlo[2]);
    constexpr int a1 = curl_a1(C), a2 = curl_a2(C);
    const double t1 = ldd<T>(a.H[a2], q) - at_minus<T>(a.H[a2], q, coord[a1], stride[a1], a.n[a1], a.per[a1]);
    const double t2 = ldd<T>(a.H[a1], q) - at_minus<T>(a.H[a1], q, coord[a2], stride[a2], a.n[a2], a.per[a2]);
    T *Ec = static_cast<T *>(a.E[C]);
    const double Eo = (double)Ec[q];
    const T *Pc_ = static_cast<const T *>(a.Pcur[C]);
    T *Pn_ = static_cast<T *>(a.Pnew[C]);
    // every term's levels are loaded before any is used, so that they stream together rather than one
    // term per memory round trip; the sum then runs over the terms in order
    T pcr[kMaxTerms], ppr[kMaxTerms];
#pragma unroll
    for (int p = 0; p < kMaxTerms; ++p) {
        if (p >= a.nterm) break;
        const bool drude = (a.drude_mask >> p) & 1;     // from the launch arguments: no load between the terms' loads
        pcr[p] = __builtin_nontemporal_load(Pc_ + (long long)p * a.mcells + m);
        ppr[p] = drude ? (T)0 : __builtin_nontemporal_load(Pn_ + (long long)p * a.mcells + m);
    }
    double pc[kMaxTerms], pp[kMaxTerms], dsum = 0.0;
#pragma unroll
    for (int p = 0; p < kMaxTerms; ++p) {
        if (p >= a.nterm) break;
        pc[p] = (double)pcr[p];
        pp[p] = (double)ppr[p];
        dsum += pc[p] - pp[p];
    }
    double amp[kMaxSources];
    load_amps(a, amp);
    const double curl = t1 - t2;
    const double En = Eo + a.inv_eps * (a.dt * curl - dsum) - source_term(a, amp, C, i, j, k);
#pragma unroll
    for (int p = 0; p < kMaxTerms; ++p) {
        if (p >= a.nterm) break;
        const double *tc = a.coef + kCoefHead + kCoefMode * p;
        const bool drude = tc[5] != 0.0;
        __builtin_nontemporal_store((T)(drude ? tc[0] * En + tc[1] * pc[p] : tc[0] * tc[6] * En - tc[1] * pc[p] - tc[2] * pp[p]),
                                    Pn_ + (long long)p * a.mcells + m);
    }
    Ec[q] = (T)En;
}

template <typename T>
__global__ __launch_bounds__(kBathBlock) void k_update_e_multi_c(const EArgs a) {
    const int nbc = gridDim.x / 3;                  // blocks per component
    const int c = blockIdx.x / nbc;
    const int t = (blockIdx.x - c * nbc) * kBathBlock + threadIdx.x;
    if (t >= a.ext[0] * a.ext12) return;
    if (c == 0) multi_component<T, 0>(a, t);
    else if (c == 1) multi_component<T, 1>(a, t);
    else multi_component<T, 2>(a, t);
}

// ---------------------------------------------------------------------------------------------
// The same update with the bath coordinates stored in 16 bits (a reduced-precision storage mode,
// reported apart from the FP32 path): YF = 1 IEEE binary16 of Y times a scale s (a power of two keeps
// the scaling exact), YF = 2 bfloat16 (the upper half of the binary32 pattern) of Y times s.  Eight
// coordinates (two mode groups) travel as one 16-byte word, so a cell's bath takes half the load
// instructions of the FP32 layout as well as half the bytes.  E and P are updated in FP64 as above; the
// bath recurrence of the scaled coordinates runs in binary32 (3.84 ms per 512^3 launch in FP64 with its
// conversions, 3.41 ms so; the error against the oracle is the format's either way) and each new value
// is rounded to the 16-bit format (round to nearest even).
// ---------------------------------------------------------------------------------------------
typedef unsigned int nv4u __attribute__((ext_vector_type(4)));

// the stored (scaled) coordinate u of a word, widened to binary32
template <int YF>
__device__ __forceinline__ float unpack16(nv4u w, int u) {
    const unsigned bits = (u & 1) ? (w[u >> 1] >> 16) : (w[u >> 1] & 0xffffu);
    if constexpr (YF == 1) return (float)__builtin_bit_cast(_Float16, (unsigned short)bits);
    return __builtin_bit_cast(float, bits << 16);
}

// a scaled coordinate (binary32) rounded to the 16-bit format
template <int YF>
__device__ __forceinline__ unsigned pack16(float f) {
    if constexpr (YF == 1) return (unsigned)__builtin_bit_cast(unsigned short, (_Float16)f);
    unsigned x = __builtin_bit_cast(unsigned, f);
    x += 0x7fffu + ((x >> 16) & 1u);                 // round to nearest even on the dropped half
    return x >> 16;
}

// NG mode groups of 4 = NG / 2 words of 8 coordinates ([word][cell] per level and component).  The
// coefficients are read from the material's FP64 table through the constant address space, the pointer
// made opaque (an empty asm) before each word's modes, so that they are re-read through the scalar cache
// where they are used instead of being held for the whole kernel: by value (166 dwords, beyond the scalar
// registers) the 512^3 bath launch took 5.42 ms, this way 4.15 ms.
template <typename T, int NG, int C, int YF>
__device__ __forceinline__ void bath_component16(const EArgs &a, int t) {
    static_assert(NG % 2 == 0, "16-bit bath words hold two mode groups");
    constexpr int NW = NG / 2;
    int i, j, k;
    unflatten<3>(t, a.lo, a.ext, a.ext12, i, j, k);
    const int s0 = a.n[1] * a.n[2], s1 = a.n[2];
    const int q = i * s0 + j * s1 + k;
    const int coord[3] = {i, j, k};
    const int stride[3] = {s0, s1, 1};
    const int m = ((i - a.mlo[0]) * a.mext[1] + (j - a.mlo[1])) * a.mext[2] + (k - a.mlo[2]);
    const int mcells = (int)a.mcells;
    constexpr int a1 = curl_a1(C), a2 = curl_a2(C);
    const bool has_sig = a.sigma != nullptr;
    const T *sp = has_sig ? static_cast<const T *>(a.sigma) + m : static_cast<const T *>(a.E[C]) + q;
    const T sig_raw = *sp;
    const double t1 = ldd<T>(a.H[a2], q) - at_minus<T>(a.H[a2], q, coord[a1], stride[a1], a.n[a1], a.per[a1]);
    const double t2 = ldd<T>(a.H[a1], q) - at_minus<T>(a.H[a1], q, coord[a2], stride[a2], a.n[a2], a.per[a2]);
    const double Eo = (double)static_cast<const T *>(a.E[C])[q];
    const double Pc = (double)__builtin_nontemporal_load(static_cast<const T *>(a.Pcur[C]) + m);
    const double Pp = (double)__builtin_nontemporal_load(static_cast<const T *>(a.Pnew[C]) + m);
    const nv4u *Yc = static_cast<const nv4u *>(a.Ycur[C]);
    nv4u *Yn = static_cast<nv4u *>(a.Ynew[C]);
    nv4u yc[NW], yp[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        yc[w] = __builtin_nontemporal_load(Yc + (long long)w * mcells + m);
        yp[w] = __builtin_nontemporal_load(Yn + (long long)w * mcells + m);
    }
    double amp[kMaxSources];
    load_amps(a, amp);
    const double sig = has_sig ? (double)sig_raw : a.sigma0;
    // the coordinates stay scaled (Y s) and their recurrence runs in binary32 (its rounding, 6e-8, is far
    // below the 16-bit format's): the FP32 block after the modes holds a_j, b_j + 1, c_j s, sa_j / s and
    // sb_j / s per mode; E and P are updated in FP64 as everywhere
    typedef const __attribute__((address_space(4))) double *cdp;
    typedef const __attribute__((address_space(4))) float *cfp;
    cdp co = (cdp)a.coef;
    const double En = Eo + a.inv_eps * (a.dt * (t1 - t2) - (Pc - Pp)) - source_term(a, amp, C, i, j, k);
    float Sf = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        asm volatile("" : "+s"(co));
        const cfp xf = (cfp)(co + kCoefHead + 4 * NG * kCoefMode) + 8 * w * 5;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            Sf += xf[u * 5 + 3] * unpack16<YF>(yc[w], u) + xf[u * 5 + 4] * unpack16<YF>(yp[w], u);
    }
    const double S = (double)Sf;
    asm volatile("" : "+s"(co));
    const double Pnew = co[0] * sig * En - co[1] * Pc - co[2] * Pp - S;
    const float dPf = (float)(Pnew - Pp);
    static_cast<T *>(a.E[C])[q] = (T)En;
    __builtin_nontemporal_store((T)Pnew, static_cast<T *>(a.Pnew[C]) + m);
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        asm volatile("" : "+s"(co));
        const cfp xf = (cfp)(co + kCoefHead + 4 * NG * kCoefMode) + 8 * w * 5;
        unsigned h[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            h[u] = pack16<YF>(xf[u * 5 + 0] * unpack16<YF>(yc[w], u) + xf[u * 5 + 1] * unpack16<YF>(yp[w], u) +
                              xf[u * 5 + 2] * dPf);
        nv4u o;
        o[0] = h[0] | (h[1] << 16);
        o[1] = h[2] | (h[3] << 16);
        o[2] = h[4] | (h[5] << 16);
        o[3] = h[6] | (h[7] << 16);
        __builtin_nontemporal_store(o, Yn + (long long)w * mcells + m);
    }
}

template <typename T, int NG, int YF>
__global__ __launch_bounds__(kBathBlock) void k_update_e_bath_c16(const EArgs a) {
    const int nbc = gridDim.x / 3;
    const int c = blockIdx.x / nbc;
    const int t = (blockIdx.x - c * nbc) * kBathBlock + threadIdx.x;
    if (t >= a.ext[0] * a.ext12) return;
    if (c == 0) bath_component16<T, NG, 0, YF>(a, t);
    else if (c == 1) bath_component16<T, NG, 1, YF>(a, t);
    else bath_component16<T, NG, 2, YF>(a, t);
}

// 16-bit bath coordinates widened to FP64 (read-out)
__global__ __launch_bounds__(kBlock) void k_bath16_to_f64(const unsigned short *src, long long n, int yf, double inv_s,
                                                          double *dst) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        const unsigned b = src[i];
        const float f = yf == 1 ? (float)__builtin_bit_cast(_Float16, (unsigned short)b) : __builtin_bit_cast(float, b << 16);
        dst[i] = (double)f * inv_s;
    }
}

hipError_t launch_bath16_to_f64(const void *src, long long n, int yf, double inv_s, double *dst, hipStream_t s) {
    const unsigned g = (unsigned)std::min<long long>((n + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(k_bath16_to_f64, dim3(g), dim3(kBlock), 0, s, (const unsigned short *)src, n, yf, inv_s, dst);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// H update, generic form
// ---------------------------------------------------------------------------------------------
template <int DIM, typename T, bool PML>
__global__ __launch_bounds__(kBlock) void k_update_h(const HArgs a) {
    RegV R;
    const int t = pick_region(a, 1.0, xcd_block(blockIdx.x, gridDim.x), R) * kBlock + threadIdx.x;
    if (t >= R.ext[0] * R.ext12) return;
    int i, j, k;
    unflatten<DIM>(t, R.lo, R.ext, R.ext12, i, j, k);
    const int s0 = a.n[1] * a.n[2], s1 = a.n[2];
    const int q = i * s0 + j * s1 + k;
    const int coord[3] = {i, j, k};
    const int stride[3] = {s0, s1, 1};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (!h_active(DIM, c)) continue;
        const int a1 = curl_a1(c), a2 = curl_a2(c);
        double t1 = 0.0, t2 = 0.0;
        if (axis_live(DIM, a1) && e_active(DIM, a2))
            t1 = at_plus_bloch<T>(a.E[a2], a.Etw[a2], q, coord[a1], stride[a1], a.n[a1], a.per[a1], a.bcos[a1],
                                  a.bsin[a1]) - ldd<T>(a.E[a2], q);
        if (axis_live(DIM, a2) && e_active(DIM, a1))
            t2 = at_plus_bloch<T>(a.E[a1], a.Etw[a1], q, coord[a2], stride[a2], a.n[a2], a.per[a2], a.bcos[a2],
                                  a.bsin[a2]) - ldd<T>(a.E[a1], q);
        if (PML) {
            if (R.psi[c][0]) {
                T *ps = static_cast<T *>(R.psi[c][0]);
                const double psi = a.pml_b[a1][coord[a1]] * (double)__builtin_nontemporal_load(ps + t) + a.pml_c[a1][coord[a1]] * t1;
                __builtin_nontemporal_store((T)psi, ps + t);
                t1 += psi;
            }
            if (R.psi[c][1]) {
                T *ps = static_cast<T *>(R.psi[c][1]);
                const double psi = a.pml_b[a2][coord[a2]] * (double)__builtin_nontemporal_load(ps + t) + a.pml_c[a2][coord[a2]] * t2;
                __builtin_nontemporal_store((T)psi, ps + t);
                t2 += psi;
            }
        }
        T *Hc = static_cast<T *>(a.H[c]);
        Hc[q] = (T)((double)Hc[q] - a.dt * (t1 - t2));
    }
}

// ---------------------------------------------------------------------------------------------
// 3D H update over a z-aligned region without CPML, four z-consecutive cells per thread:
// 16-byte loads of the own E and H rows and of the y+1 / x+1 neighbour rows, one scalar load
// for the z+1 neighbour of the last cell.
// ---------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double lane4(const vec4_t<T> &v, int e) {
    return e == 0 ? (double)v.x : e == 1 ? (double)v.y : e == 2 ? (double)v.z : (double)v.w;
}

// region of a v4 launch (always from the table) and the first of the thread's 4 z-cells
struct Cell4 {
    int i, j, k, tc;       // cell of the first z value, region-local index of that cell
    int row;               // region-local row (x, y) of a 3D cell
    bool live;
};
// Blocks in launch order, every XCD streaming next to the others: on the 512^3 grid the H pass took
// 1.02 ms against 1.06 ms, the background E pass 0.818 against 0.830 ms, with a contiguous share per XCD.
template <class A>
__device__ __forceinline__ const RegionDesc &v4_region(const A &a, Cell4 &c) {
    const int b = blockIdx.x;
    int r = -1;
#pragma unroll
    for (int s = 0; s < kMaxGroup; ++s) r += b >= a.rd->block0[s];
    const RegionDesc &D = a.rd->d[r];
    const int t = (b - a.rd->block0[r]) * kBlock + threadIdx.x;
    // the region's z range rounded out to whole 4-cell groups (a region that is not 4-aligned leaves
    // its edge groups partly outside; the kernels store only the cells inside)
    const int base = D.lo[2] & ~3;
    const int ext2q = ((D.lo[2] + D.ext[2] + 3) >> 2) - (D.lo[2] >> 2);
    c.live = t < D.ext[0] * D.ext[1] * ext2q;
    const int rr = t / ext2q;
    const int kq = t - rr * ext2q;
    const int r2 = rr / D.ext[1];
    c.k = base + 4 * kq;
    c.i = D.lo[0] + r2;
    c.j = D.lo[1] + (rr - r2 * D.ext[1]);
    c.tc = 4 * t;
    c.row = rr;
    return D;
}

// CPML convolution of one curl term for 4 z-consecutive cells: psi <- b psi + c dF, dF += psi
// Coefficients of the 4 cells: along the vector axis they differ per cell and are read as two
// 16-byte pairs (the first cell is 4-aligned, the tables 256-byte aligned); across it they are
// one value.
__device__ __forceinline__ void coef4(const double *t, bool along, int x, double *out) {
    if (along) {
        const double2 lo = *reinterpret_cast<const double2 *>(t + x);
        const double2 hi = *reinterpret_cast<const double2 *>(t + x + 2);
        out[0] = lo.x; out[1] = lo.y; out[2] = hi.x; out[3] = hi.y;
    } else {
        const double v = t[x];
        out[0] = v; out[1] = v; out[2] = v; out[3] = v;
    }
}

template <typename T>
__device__ __forceinline__ void cpml4(void *psi, int tc, int ax, int i, int j, int k, const double *pb,
                                      const double *pc, double *term) {
    using V = vec4_t<T>;
    V *pp = reinterpret_cast<V *>(static_cast<T *>(psi) + tc);
    const V p = *pp;
    const int x = ax == 0 ? i : ax == 1 ? j : k;
    double b[4], c[4], o[4];
    coef4(pb, ax == 2, x, b);
    coef4(pc, ax == 2, x, c);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        o[e] = b[e] * lane4<T>(p, e) + c[e] * term[e];
        term[e] += o[e];
    }
    V w;
    w.x = (T)o[0]; w.y = (T)o[1]; w.z = (T)o[2]; w.w = (T)o[3];
    *pp = w;
}

// The same convolution with psi already loaded (prefetched with the field rows)
template <typename T>
__device__ __forceinline__ void cpml4_apply(const vec4_t<T> &p, vec4_t<T> *pp, int k, const double *pb,
                                            const double *pc, double *term) {
    using V = vec4_t<T>;
    double b[4], c[4], o[4];
    coef4(pb, true, k, b);
    coef4(pc, true, k, c);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        o[e] = b[e] * lane4<T>(p, e) + c[e] * term[e];
        term[e] += o[e];
    }
    V w;
    w.x = (T)o[0]; w.y = (T)o[1]; w.z = (T)o[2]; w.w = (T)o[3];
    *pp = w;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_h3_v4(const HArgs a) {
    using V = vec4_t<T>;
    Cell4 C;
    const RegionDesc &D = v4_region(a, C);
    if (!C.live) return;
    const int i = C.i, j = C.j, k = C.k;
    const int s0 = a.n[1] * a.n[2], s1 = a.n[2];
    const int q = i * s0 + j * s1 + k;
    const T *Ex = static_cast<const T *>(a.E[0]);
    const T *Ey = static_cast<const T *>(a.E[1]);
    const T *Ez = static_cast<const T *>(a.E[2]);
    // neighbour rows with the axis boundary rule; an invalid neighbour reads the own row, then is zeroed
    const bool oky = j < a.n[1] - 1 || a.per[1], okx = i < a.n[0] - 1 || a.per[0], okz = k + 4 < a.n[2] || a.per[2];
    const int qy = j < a.n[1] - 1 ? q + s1 : (a.per[1] ? q - (a.n[1] - 1) * s1 : q);
    const int qx = i < a.n[0] - 1 ? q + s0 : (a.per[0] ? q - (a.n[0] - 1) * s0 : q);
    const int qz = k + 4 < a.n[2] ? q + 4 : (a.per[2] ? q + 4 - a.n[2] : q);
    const V ex = *reinterpret_cast<const V *>(Ex + q);
    const V ey = *reinterpret_cast<const V *>(Ey + q);
    const V ez = *reinterpret_cast<const V *>(Ez + q);
    const V ez_y = *reinterpret_cast<const V *>(Ez + qy);
    const V ex_y = *reinterpret_cast<const V *>(Ex + qy);
    const V ey_x = *reinterpret_cast<const V *>(Ey + qx);
    const V ez_x = *reinterpret_cast<const V *>(Ez + qx);
    // E_x and E_y one cell beyond the group: the next lane's first values when that lane holds the
    // row's next group (every lane but a row's or a wave's last), else a load
    const T exs = __shfl_down(ex.x, 1), eys = __shfl_down(ey.x, 1);
    const bool from_lane = (threadIdx.x & 63) < 63 && k + 4 < ((D.lo[2] + D.ext[2] + 3) & ~3);
    const double ex_z = from_lane ? (double)exs : (okz ? (double)Ex[qz] : 0.0);
    const double ey_z = from_lane ? (double)eys : (okz ? (double)Ey[qz] : 0.0);
    // H is read once and written once per step: streamed (non-temporal); E rows are shared with the
    // neighbouring threads and stay cacheable
    using NV = nvec4_t<T>;
    NV *Hx = reinterpret_cast<NV *>(static_cast<T *>(a.H[0]) + q);
    NV *Hy = reinterpret_cast<NV *>(static_cast<T *>(a.H[1]) + q);
    NV *Hz = reinterpret_cast<NV *>(static_cast<T *>(a.H[2]) + q);
    const NV hxn = __builtin_nontemporal_load(Hx), hyn = __builtin_nontemporal_load(Hy), hzn = __builtin_nontemporal_load(Hz);
    // z-term psi (Hx's and Hy's): per cell of the region, or (zw > 0) only for z < zlo and
    // z >= zhi, in zw slots per row (the 4-cell groups never straddle zlo or zhi); loaded here so
    // that its latency overlaps that of the field rows
    V *pz0 = nullptr, *pz1 = nullptr;
    {
        int tz = C.tc;
        bool zon = true;
        if (D.zw) {
            zon = k < D.zlo || k >= D.zhi;
            tz = C.row * D.zw + (k < D.zlo ? k - D.lo[2] : k - D.zhi + (D.zlo - D.lo[2]));
        }
        if (zon && D.psi[0][1]) pz0 = reinterpret_cast<V *>(static_cast<T *>(D.psi[0][1]) + tz);
        if (zon && D.psi[1][0]) pz1 = reinterpret_cast<V *>(static_cast<T *>(D.psi[1][0]) + tz);
    }
    V psz0{}, psz1{};
    if (pz0) psz0 = *pz0;
    if (pz1) psz1 = *pz1;
    V hx, hy, hz;
    hx.x = hxn[0]; hx.y = hxn[1]; hx.z = hxn[2]; hx.w = hxn[3];
    hy.x = hyn[0]; hy.y = hyn[1]; hy.z = hyn[2]; hy.w = hyn[3];
    hz.x = hzn[0]; hz.y = hzn[1]; hz.z = hzn[2]; hz.w = hzn[3];
    const double dt = a.dt;
    // curl terms per component: t1 along axis a1, t2 along axis a2 (Hx: y, z; Hy: z, x; Hz: x, y)
    double tx1[4], tx2[4], ty1[4], ty2[4], tz1[4], tz2[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double exe = lane4<T>(ex, e), eye = lane4<T>(ey, e), eze = lane4<T>(ez, e);
        const double exn = e < 3 ? lane4<T>(ex, e + 1) : ex_z;
        const double eyn = e < 3 ? lane4<T>(ey, e + 1) : ey_z;
        const double ezy = oky ? lane4<T>(ez_y, e) : 0.0, exy = oky ? lane4<T>(ex_y, e) : 0.0;
        const double eyx = okx ? lane4<T>(ey_x, e) : 0.0, ezx = okx ? lane4<T>(ez_x, e) : 0.0;
        tx1[e] = ezy - eze; tx2[e] = eyn - eye;
        ty1[e] = exn - exe; ty2[e] = ezx - eze;
        tz1[e] = eyx - eye; tz2[e] = exy - exe;
    }
    if (D.psi[0][0]) cpml4<T>(D.psi[0][0], C.tc, 1, i, j, k, a.pml_b[1], a.pml_c[1], tx1);
    if (pz0) cpml4_apply<T>(psz0, pz0, k, a.pml_b[2], a.pml_c[2], tx2);
    if (pz1) cpml4_apply<T>(psz1, pz1, k, a.pml_b[2], a.pml_c[2], ty1);
    if (D.psi[1][1]) cpml4<T>(D.psi[1][1], C.tc, 0, i, j, k, a.pml_b[0], a.pml_c[0], ty2);
    if (D.psi[2][0]) cpml4<T>(D.psi[2][0], C.tc, 0, i, j, k, a.pml_b[0], a.pml_c[0], tz1);
    if (D.psi[2][1]) cpml4<T>(D.psi[2][1], C.tc, 1, i, j, k, a.pml_b[1], a.pml_c[1], tz2);
    V wx, wy, wz;
    wx.x = (T)(lane4<T>(hx, 0) - dt * (tx1[0] - tx2[0])); wx.y = (T)(lane4<T>(hx, 1) - dt * (tx1[1] - tx2[1]));
    wx.z = (T)(lane4<T>(hx, 2) - dt * (tx1[2] - tx2[2])); wx.w = (T)(lane4<T>(hx, 3) - dt * (tx1[3] - tx2[3]));
    wy.x = (T)(lane4<T>(hy, 0) - dt * (ty1[0] - ty2[0])); wy.y = (T)(lane4<T>(hy, 1) - dt * (ty1[1] - ty2[1]));
    wy.z = (T)(lane4<T>(hy, 2) - dt * (ty1[2] - ty2[2])); wy.w = (T)(lane4<T>(hy, 3) - dt * (ty1[3] - ty2[3]));
    wz.x = (T)(lane4<T>(hz, 0) - dt * (tz1[0] - tz2[0])); wz.y = (T)(lane4<T>(hz, 1) - dt * (tz1[1] - tz2[1]));
    wz.z = (T)(lane4<T>(hz, 2) - dt * (tz1[2] - tz2[2])); wz.w = (T)(lane4<T>(hz, 3) - dt * (tz1[3] - tz2[3]));
    NV ox, oy, oz;
    ox[0] = wx.x; ox[1] = wx.y; ox[2] = wx.z; ox[3] = wx.w;
    oy[0] = wy.x; oy[1] = wy.y; oy[2] = wy.z; oy[3] = wy.w;
    oz[0] = wz.x; oz[1] = wz.y; oz[2] = wz.z; oz[3] = wz.w;
    __builtin_nontemporal_store(ox, Hx);
    __builtin_nontemporal_store(oy, Hy);
    __builtin_nontemporal_store(oz, Hz);
}

// ---------------------------------------------------------------------------------------------
// 2D TM (E_z, H_x, H_y) background E and H updates, four y-consecutive cells per thread (y is the
// fastest axis of a 2D grid), regions from the launch's table, CPML psi in the same pass.
// ---------------------------------------------------------------------------------------------
template <class A>
__device__ __forceinline__ const RegionDesc &v4_region2(const A &a, Cell4 &c) {
    const int b = xcd_block(blockIdx.x, gridDim.x);
    int r = -1;
#pragma unroll
    for (int s = 0; s < kMaxGroup; ++s) r += b >= a.rd->block0[s];
    const RegionDesc &D = a.rd->d[r];
    const int t = (b - a.rd->block0[r]) * kBlock + threadIdx.x;
    const int ext1q = D.ext[1] >> 2;
    c.live = t < D.ext[0] * ext1q;
    const int ii = t / ext1q;
    c.i = D.lo[0] + ii;
    c.j = D.lo[1] + 4 * (t - ii * ext1q);
    c.k = 0;
    c.tc = 4 * t;
    return D;
}

// CPML of one curl term for 4 y-consecutive cells (coefficients by axis position)
template <typename T>
__device__ __forceinline__ void cpml4y(void *psi, int tc, int ax, int i, int j, const double *pb, const double *pc,
                                       double *term) {
    using V = vec4_t<T>;
    V *pp = reinterpret_cast<V *>(static_cast<T *>(psi) + tc);
    const V p = *pp;
    const int x = ax == 0 ? i : j;
    double b[4], c[4], o[4];
    coef4(pb, ax == 1, x, b);
    coef4(pc, ax == 1, x, c);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        o[e] = b[e] * lane4<T>(p, e) + c[e] * term[e];
        term[e] += o[e];
    }
    V w;
    w.x = (T)o[0]; w.y = (T)o[1]; w.z = (T)o[2]; w.w = (T)o[3];
    *pp = w;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_e2_v4(const EArgs a) {
    using V = vec4_t<T>;
    Cell4 C;
    const RegionDesc &D = v4_region2(a, C);
    if (!C.live) return;
    const int i = C.i, j = C.j;
    const int s0 = a.n[1];
    const int q = i * s0 + j;
    const T *Hx = static_cast<const T *>(a.H[0]);
    const T *Hy = static_cast<const T *>(a.H[1]);
    const bool okx = i > 0 || a.per[0], oky = j > 0 || a.per[1];
    const int qx = i > 0 ? q - s0 : (a.per[0] ? q + (a.n[0] - 1) * s0 : q);
    const int qy = j > 0 ? q - 1 : (a.per[1] ? q + a.n[1] - 1 : q);
    const V hx = *reinterpret_cast<const V *>(Hx + q);
    const V hy = *reinterpret_cast<const V *>(Hy + q);
    const V hy_x = *reinterpret_cast<const V *>(Hy + qx);
    const double hx_y = oky ? (double)Hx[qy] : 0.0;
    V *Ez = reinterpret_cast<V *>(static_cast<T *>(a.E[2]) + q);
    const V ez = *Ez;
    // Ez: t1 = d_x Hy, t2 = d_y Hx
    double t1[4], t2[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double hxe = lane4<T>(hx, e), hye = lane4<T>(hy, e);
        t1[e] = hye - (okx ? lane4<T>(hy_x, e) : 0.0);
        t2[e] = hxe - (e > 0 ? lane4<T>(hx, e - 1) : hx_y);
    }
    if (D.psi[2][0]) cpml4y<T>(D.psi[2][0], C.tc, 0, i, j, a.pml_b[0], a.pml_c[0], t1);
    if (D.psi[2][1]) cpml4y<T>(D.psi[2][1], C.tc, 1, i, j, a.pml_b[1], a.pml_c[1], t2);
    double amp[kMaxSources];
    load_amps(a, amp);
    const double ce = a.dt * D.inv_eps;
    double o[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = lane4<T>(ez, e) + ce * (t1[e] - t2[e]) - source_term(a, amp, 2, i, j + e, 0);
    V w;
    w.x = (T)o[0]; w.y = (T)o[1]; w.z = (T)o[2]; w.w = (T)o[3];
    *Ez = w;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_h2_v4(const HArgs a) {
    using V = vec4_t<T>;
    Cell4 C;
    const RegionDesc &D = v4_region2(a, C);
    if (!C.live) return;
    const int i = C.i, j = C.j;
    const int s0 = a.n[1];
    const int q = i * s0 + j;
    const T *Ez = static_cast<const T *>(a.E[2]);
    const bool okx = i < a.n[0] - 1 || a.per[0], oky = j + 4 < a.n[1] || a.per[1];
    const int qx = i < a.n[0] - 1 ? q + s0 : (a.per[0] ? q - (a.n[0] - 1) * s0 : q);
    const int qy = j + 4 < a.n[1] ? q + 4 : (a.per[1] ? q + 4 - a.n[1] : q);
    const V ez = *reinterpret_cast<const V *>(Ez + q);
    const V ez_x = *reinterpret_cast<const V *>(Ez + qx);
    const double ez_y = oky ? (double)Ez[qy] : 0.0;
    V *Hx = reinterpret_cast<V *>(static_cast<T *>(a.H[0]) + q);
    V *Hy = reinterpret_cast<V *>(static_cast<T *>(a.H[1]) + q);
    const V hx = *Hx, hy = *Hy;
    // Hx: t1 = d_y Ez (axis y); Hy: t2 = d_x Ez (axis x), H_y <- H_y + dt t2
    double tx[4], ty[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double eze = lane4<T>(ez, e);
        tx[e] = (e < 3 ? lane4<T>(ez, e + 1) : ez_y) - eze;
        ty[e] = (okx ? lane4<T>(ez_x, e) : 0.0) - eze;
    }
    if (D.psi[0][0]) cpml4y<T>(D.psi[0][0], C.tc, 1, i, j, a.pml_b[1], a.pml_c[1], tx);
    if (D.psi[1][1]) cpml4y<T>(D.psi[1][1], C.tc, 0, i, j, a.pml_b[0], a.pml_c[0], ty);
    const double dt = a.dt;
    V wx, wy;
    wx.x = (T)(lane4<T>(hx, 0) - dt * tx[0]); wx.y = (T)(lane4<T>(hx, 1) - dt * tx[1]);
    wx.z = (T)(lane4<T>(hx, 2) - dt * tx[2]); wx.w = (T)(lane4<T>(hx, 3) - dt * tx[3]);
    wy.x = (T)(lane4<T>(hy, 0) + dt * ty[0]); wy.y = (T)(lane4<T>(hy, 1) + dt * ty[1]);
    wy.z = (T)(lane4<T>(hy, 2) + dt * ty[2]); wy.w = (T)(lane4<T>(hy, 3) + dt * ty[3]);
    *Hx = wx;
    *Hy = wy;
}

// ---------------------------------------------------------------------------------------------
// 3D E update of background regions (vacuum, dielectric, CPML) or of Drude regions (DRUDE: the
// polarization increment V = P^{n+1/2} - P^{n-1/2} read and written in the same pass, each region's
// material from the table), four z-consecutive cells per thread, regions from the launch's table
// (no energy sampling: launches with monitors take the generic kernel).
// ---------------------------------------------------------------------------------------------
template <typename T, bool DRUDE>
__global__ __launch_bounds__(kBlock) void k_update_e3_v4(const EArgs a) {
    using V = vec4_t<T>;
    Cell4 C;
    const RegionDesc &D = v4_region(a, C);
    if (!C.live) return;
    const int i = C.i, j = C.j, k = C.k;
    const int s0 = a.n[1] * a.n[2], s1 = a.n[2];
    const int q = i * s0 + j * s1 + k;
    const T *Hx = static_cast<const T *>(a.H[0]);
    const T *Hy = static_cast<const T *>(a.H[1]);
    const T *Hz = static_cast<const T *>(a.H[2]);
    const bool oky = j > 0 || a.per[1], okx = i > 0 || a.per[0], okz = k > 0 || a.per[2];
    const int qy = j > 0 ? q - s1 : (a.per[1] ? q + (a.n[1] - 1) * s1 : q);
    const int qx = i > 0 ? q - s0 : (a.per[0] ? q + (a.n[0] - 1) * s0 : q);
    const int qz = k > 0 ? q - 1 : (a.per[2] ? q + a.n[2] - 1 : q);
    const V hx = *reinterpret_cast<const V *>(Hx + q);
    const V hy = *reinterpret_cast<const V *>(Hy + q);
    const V hz = *reinterpret_cast<const V *>(Hz + q);
    const V hz_y = *reinterpret_cast<const V *>(Hz + qy);
    const V hx_y = *reinterpret_cast<const V *>(Hx + qy);
    const V hy_x = *reinterpret_cast<const V *>(Hy + qx);
    const V hz_x = *reinterpret_cast<const V *>(Hz + qx);
    // H_x and H_y one cell before the group: the previous lane's last values when that lane holds
    // the row's previous group, else a load
    const T hxs = __shfl_up(hx.w, 1), hys = __shfl_up(hy.w, 1);
    const bool from_lane = (threadIdx.x & 63) > 0 && k > (D.lo[2] & ~3);
    const double hx_z = from_lane ? (double)hxs : (okz ? (double)Hx[qz] : 0.0);
    const double hy_z = from_lane ? (double)hys : (okz ? (double)Hy[qz] : 0.0);
    // E is read once and written once per step: streamed (non-temporal); H rows are shared with the
    // neighbouring threads and stay cacheable
    using NV = nvec4_t<T>;
    NV *Ex = reinterpret_cast<NV *>(static_cast<T *>(a.E[0]) + q);
    NV *Ey = reinterpret_cast<NV *>(static_cast<T *>(a.E[1]) + q);
    NV *Ez = reinterpret_cast<NV *>(static_cast<T *>(a.E[2]) + q);
    const NV exn = __builtin_nontemporal_load(Ex), eyn = __builtin_nontemporal_load(Ey), ezn = __builtin_nontemporal_load(Ez);
    // the Drude increments and the z-term psi (Ex's, Ey's) are loaded with the field rows, so that
    // their latency overlaps
    NV vv[3];
    const int m = DRUDE ? ((i - D.mlo[0]) * D.mext[1] + (j - D.mlo[1])) * D.mext[2] + (k - D.mlo[2]) : 0;
    if (DRUDE) {
#pragma unroll
        for (int c = 0; c < 3; ++c) vv[c] = __builtin_nontemporal_load(reinterpret_cast<const NV *>(static_cast<const T *>(D.V[c]) + m));
    }
    V *pz0 = D.psi[0][1] ? reinterpret_cast<V *>(static_cast<T *>(D.psi[0][1]) + C.tc) : nullptr;
    V *pz1 = D.psi[1][0] ? reinterpret_cast<V *>(static_cast<T *>(D.psi[1][0]) + C.tc) : nullptr;
    V psz0{}, psz1{};
    if (pz0) psz0 = *pz0;
    if (pz1) psz1 = *pz1;
    V ex, ey, ez;
    ex.x = exn[0]; ex.y = exn[1]; ex.z = exn[2]; ex.w = exn[3];
    ey.x = eyn[0]; ey.y = eyn[1]; ey.z = eyn[2]; ey.w = eyn[3];
    ez.x = ezn[0]; ez.y = ezn[1]; ez.z = ezn[2]; ez.w = ezn[3];
    // Ex: t1 = d_y Hz, t2 = d_z Hy;  Ey: t1 = d_z Hx, t2 = d_x Hz;  Ez: t1 = d_x Hy, t2 = d_y Hx
    double tx1[4], tx2[4], ty1[4], ty2[4], tz1[4], tz2[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double hxe = lane4<T>(hx, e), hye = lane4<T>(hy, e), hze = lane4<T>(hz, e);
        const double hxp = e > 0 ? lane4<T>(hx, e - 1) : hx_z;
        const double hyp = e > 0 ? lane4<T>(hy, e - 1) : hy_z;
        const double hzy = oky ? lane4<T>(hz_y, e) : 0.0, hxy = oky ? lane4<T>(hx_y, e) : 0.0;
        const double hyx = okx ? lane4<T>(hy_x, e) : 0.0, hzx = okx ? lane4<T>(hz_x, e) : 0.0;
        tx1[e] = hze - hzy; tx2[e] = hye - hyp;
        ty1[e] = hxe - hxp; ty2[e] = hze - hzx;
        tz1[e] = hye - hyx; tz2[e] = hxe - hxy;
    }
    if (D.psi[0][0]) cpml4<T>(D.psi[0][0], C.tc, 1, i, j, k, a.pml_b[1], a.pml_c[1], tx1);
    if (pz0) cpml4_apply<T>(psz0, pz0, k, a.pml_b[2], a.pml_c[2], tx2);
    if (pz1) cpml4_apply<T>(psz1, pz1, k, a.pml_b[2], a.pml_c[2], ty1);
    if (D.psi[1][1]) cpml4<T>(D.psi[1][1], C.tc, 0, i, j, k, a.pml_b[0], a.pml_c[0], ty2);
    if (D.psi[2][0]) cpml4<T>(D.psi[2][0], C.tc, 0, i, j, k, a.pml_b[0], a.pml_c[0], tz1);
    if (D.psi[2][1]) cpml4<T>(D.psi[2][1], C.tc, 1, i, j, k, a.pml_b[1], a.pml_c[1], tz2);
    double amp[kMaxSources];
    load_amps(a, amp);
    const double ce = a.dt * D.inv_eps;
    double ox[4], oy[4], oz[4];
    if (DRUDE) {
        // Drude: E^{n+1/2} = E^{n-1/2} + (dt curl H - V) / eps - dt J / eps;  V' = dE E^{n+1/2} + dV V
        const double dE = D.coef[0], dV = D.coef[1];
        double *o3[3] = {ox, oy, oz};
        const V *ev[3] = {&ex, &ey, &ez};
        double *t1s[3] = {tx1, ty1, tz1}, *t2s[3] = {tx2, ty2, tz2};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            nvec4_t<T> *Vp = reinterpret_cast<nvec4_t<T> *>(static_cast<T *>(D.V[c]) + m);
            nvec4_t<T> vn;
            double vo[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double v = (double)vv[c][e];
                o3[c][e] = lane4<T>(*ev[c], e) + D.inv_eps * (a.dt * (t1s[c][e] - t2s[c][e]) - v) -
                           source_term(a, amp, c, i, j, k + e);
                vo[e] = dE * o3[c][e] + dV * v;
            }
            vn[0] = (T)vo[0]; vn[1] = (T)vo[1]; vn[2] = (T)vo[2]; vn[3] = (T)vo[3];
            __builtin_nontemporal_store(vn, Vp);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            ox[e] = lane4<T>(ex, e) + ce * (tx1[e] - tx2[e]) - source_term(a, amp, 0, i, j, k + e);
            oy[e] = lane4<T>(ey, e) + ce * (ty1[e] - ty2[e]) - source_term(a, amp, 1, i, j, k + e);
            oz[e] = lane4<T>(ez, e) + ce * (tz1[e] - tz2[e]) - source_term(a, amp, 2, i, j, k + e);
        }
    }
    NV wx, wy, wz;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        wx[e] = (T)ox[e];
        wy[e] = (T)oy[e];
        wz[e] = (T)oz[e];
    }
    const int klo = D.lo[2], khi = D.lo[2] + D.ext[2];
    if (k >= klo && k + 4 <= khi) {
        __builtin_nontemporal_store(wx, Ex);
        __builtin_nontemporal_store(wy, Ey);
        __builtin_nontemporal_store(wz, Ez);
    } else {   // edge group of a region that is not 4-aligned (background cells only): own cells only
        T *ex_ = static_cast<T *>(a.E[0]) + q, *ey_ = static_cast<T *>(a.E[1]) + q, *ez_ = static_cast<T *>(a.E[2]) + q;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (k + e >= klo && k + e < khi) {
                ex_[e] = wx[e];
                ey_[e] = wy[e];
                ez_[e] = wz[e];
            }
    }
}

// ---------------------------------------------------------------------------------------------
// clock, energy reduction, DFT, watchdog
// ---------------------------------------------------------------------------------------------
__global__ void k_tick(Clock *clk, const SourceDev *src, int nsrc, double dt) {
    const long long n = clk->next;
    __syncthreads();
    const int s = threadIdx.x;
    if (s < nsrc) {
        const SourceDev &S = src[s];
        const double tn = (double)n * dt;
        double J = 0.0;
        if (!(tn > 2.0 * S.t0)) {
            const double u = tn - S.t0;
            J = S.amplitude * exp(-u * u / (2.0 * S.tau * S.tau)) * cos(S.omega_c * u);
        }
        clk->amp[s] = J;
    }
    if (s == 0) { clk->step = n; clk->next = n + 1; }
}

// sum the block partials of one monitor into out[sample][3] on sample steps
__global__ __launch_bounds__(kBlock) void k_energy_reduce(const Clock *clk, const double *partial, long long nslots,
                                                         int every, double *out, long long capacity) {
    const long long st = clk->step;
    if (st % every) return;
    const long long sidx = st / every;
    if (sidx >= capacity) return;
    double a = 0.0, b = 0.0, c = 0.0;
    for (long long s = threadIdx.x; s < nslots; s += kBlock) {
        a += partial[3 * s]; b += partial[3 * s + 1]; c += partial[3 * s + 2];
    }
    block_sum3(a, b, c);
    if (threadIdx.x == 0) { out[3 * sidx] = a; out[3 * sidx + 1] = b; out[3 * sidx + 2] = c; }
}



template <typename T>
__global__ __launch_bounds__(kBlock) void k_dft_stage(const DftArgs a) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= a.npts) return;
    int r = p / a.ext[2];
    const int k = a.lo[2] + (p - r * a.ext[2]);
    const int r2 = r / a.ext[1];
    const int i = a.lo[0] + r2, j = a.lo[1] + (r - r2 * a.ext[1]);
    const long long s0 = (long long)a.n[1] * a.n[2], s1 = a.n[2];
    const long long q = i * s0 + j * s1 + k;
    const int coord[3] = {i, j, k};
    const long long stride[3] = {s0, s1, 1};
    const int ax = a.axis;
    double *st = a.stage + (long long)a.slot * 4 * a.npts;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        st[(long long)u * a.npts + p] = a.E[u] ? ldd<T>(a.E[u], q) : 0.0;
        double h = 0.0;
        if (a.H[u]) h = 0.5 * (at_minus<T>(a.H[u], q, coord[ax], stride[ax], a.n[ax], a.per[ax]) + ldd<T>(a.H[u], q));
        st[(long long)(2 + u) * a.npts + p] = h;
    }
}

// twiddles tw[slot][f] = dt (cos, sin) of w_f t for E times (n+1/2) dt and H times (n+1) dt
__global__ void k_dft_twiddle(const Clock *clk, const double *omega, int nf, int nslots, double dt, double *tw) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nf * nslots) return;
    const int b = id / nf, f = id - b * nf;
    const long long step = clk->step - (nslots - 1) + b;
    const double tE = ((double)step + 0.5) * dt, tH = ((double)step + 1.0) * dt;
    double sE, cE, sH, cH;
    sincos(omega[f] * tE, &sE, &cE);
    sincos(omega[f] * tH, &sH, &cH);
    double *o = tw + 4 * (long long)id;
    o[0] = dt * cE; o[1] = dt * sE; o[2] = dt * cH; o[3] = dt * sH;
}

// acc[field][f][p] += sum_b stage[b][field][p] * tw[b][f]
// One thread per (plane point, field): its staged samples are read once and held in registers, and
// the frequencies are swept in chunks whose twiddles sit in LDS (register tiles of kFlushTile
// frequencies, whose accumulators are loaded before their sums are formed, so that the loads overlap
// the arithmetic).  Each accumulator is read and written once per flush, and each sum runs over the
// slots in order, as a plain loop would.  (Before: one launch dimension per 32-frequency tile, the samples
// read again for every tile: 12.9 GB moved per flush of the 512^2 plane against 9.1 GB; 3.75 ms per flush
// then, 3.74 ms with the samples read once, 2.90 ms with the accumulator loads issued ahead, 2.83 ms with
// 64-frequency chunks; 4-frequency register tiles 2.92 ms.)
constexpr int kFlushChunk = 64;      // frequencies whose twiddles are in LDS at once (64 KB)
constexpr int kFlushTile = 8;        // frequencies accumulated in registers at once
__global__ __launch_bounds__(kBlock) void k_dft_flush(const double *stage, const double *tw, int npts, int nf,
                                                     int nslots, double2 *acc) {
    __shared__ double2 ltw[kDftSlots][kFlushChunk];
    const int field = blockIdx.y;
    const int hsel = field >= 2 ? 2 : 0;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    const bool live = p < npts;
    double x[kDftSlots];
#pragma unroll
    for (int b = 0; b < kDftSlots; ++b)
        x[b] = (live && b < nslots) ? __builtin_nontemporal_load(stage + ((long long)b * 4 + field) * npts + p) : 0.0;
    for (int c0 = 0; c0 < nf; c0 += kFlushChunk) {
        __syncthreads();                             // the previous chunk's twiddles are read by now
        for (int id = threadIdx.x; id < nslots * kFlushChunk; id += kBlock) {
            const int b = id / kFlushChunk, f = id - b * kFlushChunk;
            double2 v = make_double2(0.0, 0.0);
            if (c0 + f < nf) {
                const double *o = tw + 4 * ((long long)b * nf + c0 + f);
                v = make_double2(o[hsel], o[hsel + 1]);
            }
            ltw[b][f] = v;
        }
        __syncthreads();
        if (!live) continue;
        for (int t0 = 0; t0 < kFlushChunk && c0 + t0 < nf; t0 += kFlushTile) {
            double re[kFlushTile], im[kFlushTile];
            double2 av[kFlushTile];
#pragma unroll
            for (int f = 0; f < kFlushTile; ++f) {
                re[f] = 0.0; im[f] = 0.0;
                av[f] = c0 + t0 + f < nf ? acc[((long long)field * nf + c0 + t0 + f) * npts + p] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int b = 0; b < kDftSlots; ++b) {
                if (b < nslots) {
#pragma unroll
                    for (int f = 0; f < kFlushTile; ++f) {
                        re[f] += x[b] * ltw[b][t0 + f].x;
                        im[f] += x[b] * ltw[b][t0 + f].y;
                    }
                }
            }
#pragma unroll
            for (int f = 0; f < kFlushTile; ++f) {
                if (c0 + t0 + f >= nf) continue;
                double2 *d = acc + ((long long)field * nf + c0 + t0 + f) * npts + p;
                double2 v = av[f];
                v.x += re[f];
                v.y += im[f];
                *d = v;
            }
        }
    }
}

// flux[f] = Re sum_p (E1 conj(H2) - E2 conj(H1)).  Bloch pair (acc_im != nullptr): the transforms are
// those of the complex fields, acc + i acc_im (acc, acc_im: the real and imaginary parts' transforms).
__device__ __forceinline__ double2 dft_value(const double2 *acc, const double2 *acc_im, long long i) {
    double2 v = acc[i];
    if (acc_im) {
        const double2 w = acc_im[i];
        v.x -= w.y;
        v.y += w.x;
    }
    return v;
}
__global__ __launch_bounds__(kBlock) void k_dft_flux(const double2 *acc, const double2 *acc_im, int npts, int nf,
                                                     double *flux) {
    const int f = blockIdx.x;
    const long long o1 = (0LL * nf + f) * npts, o2 = (1LL * nf + f) * npts;
    const long long o3 = (2LL * nf + f) * npts, o4 = (3LL * nf + f) * npts;
    double s = 0.0, z1 = 0.0, z2 = 0.0;
    for (int p = threadIdx.x; p < npts; p += kBlock) {
        const double2 e1 = dft_value(acc, acc_im, o1 + p), e2 = dft_value(acc, acc_im, o2 + p);
        const double2 h1 = dft_value(acc, acc_im, o3 + p), h2 = dft_value(acc, acc_im, o4 + p);
        s += (e1.x * h2.x + e1.y * h2.y) - (e2.x * h1.x + e2.y * h1.y);
    }
    block_sum3(s, z1, z2);
    if (threadIdx.x == 0) flux[f] = s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_nonfinite(const T *f, long long n, int *flag) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        const double v = (double)f[i];
        if (!(v == v) || v - v != 0.0) { atomicOr(flag, 1); return; }
    }
}

// a field in its storage type widened to FP64 into a device buffer (device-side read-out)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_f64(const T *f, long long n, double *out) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        out[i] = (double)f[i];
}

// trajectory recorder: row n of the record = step n (steps beyond the capacity are not recorded)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_probe(const T *E, const T *P, const int *q, const int *m, int n,
                                                  const Clock *clk, long long capacity, float *outE, float *outP) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const long long row = clk->step;
    if (i >= n || row >= capacity) return;
    outE[row * n + i] = (float)E[q[i]];
    outP[row * n + i] = (float)P[m[i]];
}

// ---------------------------------------------------------------------------------------------
// launchers (host side)
// ---------------------------------------------------------------------------------------------
static inline unsigned nblocks(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <int DIM, typename T, int KIND, int NG, bool PML>
static hipError_t launch_e_pml(const EArgs &a, const double *coef_host, bool energy, hipStream_t s) {
    const long long n = (long long)a.ext[0] * a.ext12;
    if (n == 0) return hipSuccess;
    constexpr int NC = DIM == 3 ? 3 : 1;
    // of the specialised bath kernels only the 2D load-first one reads the other part of a Bloch pair
    // (the wrap rows; other launches of a pair are real-grid launches); of them only the component-split
    // kernel carries the thermal / anharmonic terms (without energy sampling), other extended baths take
    // k_update_e
    if constexpr (KIND == K_BATH && !PML && NG > 0 && NC * NG <= 16 && DIM == 3 && NC * NG > 6) {
        if (!a.bloch && a.bext && !energy) {
            // no occupancy cap: with the noise generator the kernel is bound by its arithmetic as much as by
            // its bytes and runs best at its register limit of 3 waves per SIMD (512^3 layer 6.26 ms,
            // 7.45 ms at 2.5 waves, 9.37 ms at 2; bounding it to 4 waves would spill 47 registers)
            BathCoef<NG> cf{};
            hipLaunchKernelGGL((k_update_e_bath_c<T, NG, true>), dim3(3 * (unsigned)((n + kBathBlock - 1) / kBathBlock)),
                               dim3(kBathBlock), 0, s, a, cf);
            return hipGetLastError();
        }
    }
    if constexpr (KIND == K_BATH && !PML && NG > 0 && NC * NG <= 16) {
        if ((!a.bloch || DIM == 2) && !a.bext) {
            BathCoef<NG> cf;
            for (int h = 0; h < 3; ++h) cf.head[h] = coef_host[h];
            for (int j = 0; j < 4 * NG; ++j)
                for (int u = 0; u < 5; ++u) cf.md[j][u] = coef_host[kCoefHead + j * kCoefMode + u];
            if (energy)
                hipLaunchKernelGGL((k_update_e_bath<DIM, T, NG, true>), dim3(nblocks(n)), dim3(kBlock), 0, s, a, cf);
            else if constexpr (DIM == 3 && NC * NG > 6) {
                const dim3 grid(3 * (unsigned)((n + kBathBlock - 1) / kBathBlock));
                if constexpr (std::is_same<T, float>::value && NG % 2 == 0) {
                    if (a.yfmt == 1) {
                        hipLaunchKernelGGL((k_update_e_bath_c16<T, NG, 1>), grid, dim3(kBathBlock), 0, s, a);
                        return hipGetLastError();
                    }
                    if (a.yfmt == 2) {
                        hipLaunchKernelGGL((k_update_e_bath_c16<T, NG, 2>), grid, dim3(kBathBlock), 0, s, a);
                        return hipGetLastError();
                    }
                }
                hipLaunchKernelGGL((k_update_e_bath_c<T, NG, false>), grid, dim3(kBathBlock), kBathLdsReserve, s, a, cf);
            }
            else
                hipLaunchKernelGGL((k_update_e_bath<DIM, T, NG, false>),
                                   dim3(nblocks(DIM == 3 ? pair_threads(a.ext) : n)), dim3(kBlock), 0, s, a, cf);
            return hipGetLastError();
        }
    }
    if constexpr (KIND == K_MULTI && DIM == 3 && !PML) {
        if (!a.bloch && !energy) {
            hipLaunchKernelGGL(k_update_e_multi_c<T>, dim3(3 * (unsigned)((n + kBathBlock - 1) / kBathBlock)),
                               dim3(kBathBlock), 0, s, a);
            return hipGetLastError();
        }
    }
    if constexpr (KIND == K_BATH && NG > 0 && !PML) {
        if (a.bext) {
            if (energy)
                hipLaunchKernelGGL((k_update_e<DIM, T, KIND, NG, PML, true, true>), dim3(nblocks(n)), dim3(kBlock), 0, s, a);
            else
                hipLaunchKernelGGL((k_update_e<DIM, T, KIND, NG, PML, false, true>), dim3(nblocks(n)), dim3(kBlock), 0, s, a);
            return hipGetLastError();
        }
    }
    if (energy)
        hipLaunchKernelGGL((k_update_e<DIM, T, KIND, NG, PML, true>), dim3(nblocks(n)), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_update_e<DIM, T, KIND, NG, PML, false>), dim3(nblocks(n)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int DIM, typename T>
static hipError_t launch_e_dim(const EArgs &a, const double *ch, int kind, int ng, bool pml, bool energy, hipStream_t s) {
    if (DIM == 2 && kind == K_BACKGROUND && a.nrd < 0) {   // y-vectorized 2D launch over the table's regions
        const long long n = (long long)a.ext[0] * a.ext12;
        if (n == 0) return hipSuccess;
        hipLaunchKernelGGL(k_update_e2_v4<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    if (DIM == 3 && (kind == K_BACKGROUND || kind == K_DRUDE) && a.nrd < 0) {   // z-vectorized launch
        const long long n = (long long)a.ext[0] * a.ext12;
        if (n == 0) return hipSuccess;
        if (kind == K_DRUDE)
            hipLaunchKernelGGL((k_update_e3_v4<T, true>), dim3(nblocks(n)), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_update_e3_v4<T, false>), dim3(nblocks(n)), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    if (kind == K_BACKGROUND)
        return pml ? launch_e_pml<DIM, T, K_BACKGROUND, 0, true>(a, ch, energy, s)
                   : launch_e_pml<DIM, T, K_BACKGROUND, 0, false>(a, ch, energy, s);
    if (kind == K_DRUDE) return launch_e_pml<DIM, T, K_DRUDE, 0, false>(a, ch, energy, s);
    if (kind == K_MULTI) return launch_e_pml<DIM, T, K_MULTI, 0, false>(a, ch, energy, s);
    if (kind == K_CLOSURE) {
        const long long n = (long long)a.ext[0] * a.ext12;
        if (n == 0) return hipSuccess;
        if (energy)
            hipLaunchKernelGGL((k_update_e_closure<DIM, T, true>), dim3(nblocks(n)), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_update_e_closure<DIM, T, false>), dim3(nblocks(n)), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    if (kind == K_BATH) {
        switch (ng) {
            case 0: return launch_e_pml<DIM, T, K_BATH, 0, false>(a, ch, energy, s);
            case 1: return launch_e_pml<DIM, T, K_BATH, 1, false>(a, ch, energy, s);
            case 2: return launch_e_pml<DIM, T, K_BATH, 2, false>(a, ch, energy, s);
            case 3: return launch_e_pml<DIM, T, K_BATH, 3, false>(a, ch, energy, s);
            case 4: return launch_e_pml<DIM, T, K_BATH, 4, false>(a, ch, energy, s);
            case 6: return launch_e_pml<DIM, T, K_BATH, 6, false>(a, ch, energy, s);
            case 8: return launch_e_pml<DIM, T, K_BATH, 8, false>(a, ch, energy, s);
            case 12: return launch_e_pml<DIM, T, K_BATH, 12, false>(a, ch, energy, s);
            case 16: return launch_e_pml<DIM, T, K_BATH, 16, false>(a, ch, energy, s);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_probe(bool f64, const void *E, const void *P, const int *q, const int *m, int n, const Clock *clk,
                        long long capacity, float *outE, float *outP, hipStream_t s) {
    if (f64)
        hipLaunchKernelGGL(k_probe<double>, dim3(nblocks(n)), dim3(kBlock), 0, s, (const double *)E, (const double *)P, q,
                           m, n, clk, capacity, outE, outP);
    else
        hipLaunchKernelGGL(k_probe<float>, dim3(nblocks(n)), dim3(kBlock), 0, s, (const float *)E, (const float *)P, q, m,
                           n, clk, capacity, outE, outP);
    return hipGetLastError();
}

hipError_t launch_update_e(int dim, bool f64, const EArgs &a, const double *coef_host, int kind, int ng, bool pml,
                           bool energy, hipStream_t s) {
    if (f64) {
        if (dim == 1) return launch_e_dim<1, double>(a, coef_host, kind, ng, pml, energy, s);
        if (dim == 2) return launch_e_dim<2, double>(a, coef_host, kind, ng, pml, energy, s);
        return launch_e_dim<3, double>(a, coef_host, kind, ng, pml, energy, s);
    }
    if (dim == 1) return launch_e_dim<1, float>(a, coef_host, kind, ng, pml, energy, s);
    if (dim == 2) return launch_e_dim<2, float>(a, coef_host, kind, ng, pml, energy, s);
    return launch_e_dim<3, float>(a, coef_host, kind, ng, pml, energy, s);
}

template <int DIM, typename T>
static hipError_t launch_h_dim(const HArgs &a, bool pml, hipStream_t s) {
    const long long n = (long long)a.ext[0] * a.ext12;
    if (n == 0) return hipSuccess;
    if (DIM == 3 && a.nrd < 0) {       // z-vectorized launch: the table holds the regions, ext[0] the threads
        hipLaunchKernelGGL(k_update_h3_v4<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    if (DIM == 2 && a.nrd < 0) {       // y-vectorized 2D launch
        hipLaunchKernelGGL(k_update_h2_v4<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    if (pml)
        hipLaunchKernelGGL((k_update_h<DIM, T, true>), dim3(nblocks(n)), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_update_h<DIM, T, false>), dim3(nblocks(n)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_update_h(int dim, bool f64, const HArgs &a, bool pml, hipStream_t s) {
    if (f64) {
        if (dim == 1) return launch_h_dim<1, double>(a, pml, s);
        if (dim == 2) return launch_h_dim<2, double>(a, pml, s);
        return launch_h_dim<3, double>(a, pml, s);
    }
    if (dim == 1) return launch_h_dim<1, float>(a, pml, s);
    if (dim == 2) return launch_h_dim<2, float>(a, pml, s);
    return launch_h_dim<3, float>(a, pml, s);
}

hipError_t launch_tick(Clock *clk, const SourceDev *src, int nsrc, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, clk, src, nsrc, dt);
    return hipGetLastError();
}

hipError_t launch_energy_reduce(const Clock *clk, const double *partial, long long nslots, int every, double *out,
                                long long capacity, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_reduce, dim3(1), dim3(kBlock), 0, s, clk, partial, nslots, every, out, capacity);
    return hipGetLastError();
}

hipError_t launch_dft_stage(bool f64, const DftArgs &a, hipStream_t s) {
    if (f64)
        hipLaunchKernelGGL(k_dft_stage<double>, dim3(nblocks(a.npts)), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_dft_stage<float>, dim3(nblocks(a.npts)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_dft_flush(const Clock *clk, const double *omega, int nf, int nslots, double dt, double *tw,
                            const double *stage, int npts, double2 *acc, hipStream_t s) {
    const int ntw = nf * nslots;
    hipLaunchKernelGGL(k_dft_twiddle, dim3((ntw + 255) / 256), dim3(256), 0, s, clk, omega, nf, nslots, dt, tw);
    hipLaunchKernelGGL(k_dft_flush, dim3(nblocks(npts), 4), dim3(kBlock), 0, s, stage, tw, npts, nf, nslots, acc);
    return hipGetLastError();
}

hipError_t launch_dft_flux(const double2 *acc, const double2 *acc_im, int npts, int nf, double *flux, hipStream_t s) {
    hipLaunchKernelGGL(k_dft_flux, dim3(nf), dim3(kBlock), 0, s, acc, acc_im, npts, nf, flux);
    return hipGetLastError();
}

hipError_t launch_to_f64(bool f64, const void *src, long long n, double *dst, hipStream_t s) {
    const unsigned g = (unsigned)std::min<long long>((n + kBlock - 1) / kBlock, 8192);
    if (f64)
        hipLaunchKernelGGL(k_to_f64<double>, dim3(g), dim3(kBlock), 0, s, (const double *)src, n, dst);
    else
        hipLaunchKernelGGL(k_to_f64<float>, dim3(g), dim3(kBlock), 0, s, (const float *)src, n, dst);
    return hipGetLastError();
}

hipError_t launch_nonfinite(bool f64, const void *f, long long n, int *flag, hipStream_t s) {
    const unsigned g = (unsigned)std::min<long long>((n + kBlock - 1) / kBlock, 4096);
    if (f64)
        hipLaunchKernelGGL(k_nonfinite<double>, dim3(g), dim3(kBlock), 0, s, (const double *)f, n, flag);
    else
        hipLaunchKernelGGL(k_nonfinite<float>, dim3(g), dim3(kBlock), 0, s, (const float *)f, n, flag);
    return hipGetLastError();
}

}  // namespace fdtdb
