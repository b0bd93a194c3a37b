// Internal types shared by the host runtime and the HIP kernels of libfdtdb.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdtdb {

constexpr int kMaxSources = 4;
constexpr int kMaxModes = 64;
constexpr int kMaxEnergy = 4;
constexpr int kBlock = 256;          // threads per block of the stencil kernels
// Component-split 3D bath kernel: 128-thread blocks, at most 4 of them per CU (2 waves per SIMD), held
// there by an LDS reservation the kernel does not use (4 x 36 KiB fit the 160 KiB of a CU, 5 do not).  Its
// registers allow 4 waves per SIMD, but it streams best with fewer requests in flight: on the 512^3 layer
// with N_b = 16 (coefficients through scalar loads) 5.77 ms per launch at 2 waves, 5.98 at 2.5, 6.05 at
// 3, 6.10 at 3.5, 6.21 at 4 (before the scalar-load coefficients: 6.10 at 2.5 and 3 waves, 6.27 at 4).
constexpr int kBathBlock = 128;
constexpr unsigned kBathLdsReserve = 36 * 1024;
constexpr int kDftSlots = 64;        // steps staged before a DFT flush

// Update kind of a region.
enum Kind : int { K_BACKGROUND = 0, K_DRUDE = 1, K_BATH = 2, K_CLOSURE = 3, K_MULTI = 4 };
constexpr int kMaxTerms = 8;          // Lorentz / Drude terms of one multi-term material

// Learned bath closure: 7 inputs -> tanh(32) -> tanh(32) -> 5 outputs.  Weight layout (row major):
// W1[32][7], b1[32], W2[32][32], b2[32], W3[5][32], b3[5].
constexpr int kClosureWidth = 32;
constexpr int kClosureParams = 32 * 7 + 32 + 32 * 32 + 32 + 5 * 32 + 5;

// Position of weight e in the transposed copy kept next to the weights: W1T[7][32], b1, W2T[32][32],
// b2, W3T[32][5], b3 (same block offsets).  Loops over an input feature with all output units as
// independent accumulators read one contiguous row of the transposed copy per feature.
__host__ __device__ inline int closure_tpos(int e) {
    constexpr int W = 32, B1 = W * 7, W2 = B1 + W, B2 = W2 + W * W, W3 = B2 + W, B3 = W3 + 5 * W;
    if (e < B1) return (e % 7) * W + e / 7;
    if (e >= W2 && e < B2) return W2 + ((e - W2) % W) * W + (e - W2) / W;
    if (e >= W3 && e < B3) return W3 + ((e - W3) % W) * 5 + (e - W3) / W;
    return e;
}

// tanh in FP32: odd Taylor series below |a| = 1/16 (no transcendental; a wave whose lanes are all
// in range skips the exponential), 1 - 2 / (1 + e^{2a}) above (absolute error about 1e-7;
// saturates to +-1 for large |a|).  Shared by closure inference and training.
__device__ __forceinline__ float tanh_f(float a) {
    if (fabsf(a) < 0.0625f) {
        const float a2 = a * a;
        return a * (1.0f + a2 * (-1.0f / 3.0f + a2 * (2.0f / 15.0f)));
    }
    return 1.0f - 2.0f / (1.0f + __expf(2.0f * a));
}

// tanh of N values with one branch per wave on the largest |a| of all lanes: below 2^-12 tanh(a) = a to
// FP32 rounding (the cubic term is under half an ulp); below 2^-7 two series terms (relative error
// 2a^4/15 < 1e-9); below 1/16 three terms (the same values as tanh_f); otherwise the exponential form.
template <int N>
__device__ __forceinline__ void tanh_n(float *v) {
    float mx = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) mx = fmaxf(mx, fabsf(v[i]));
    if (__all(mx < 0x1p-12f)) return;
    if (__all(mx < 0x1p-7f)) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = fmaf(v[i] * v[i] * (-1.0f / 3.0f), v[i], v[i]);
        return;
    }
    if (__all(mx < 0.0625f)) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const float a2 = v[i] * v[i];
            v[i] = v[i] * (1.0f + a2 * (-1.0f / 3.0f + a2 * (2.0f / 15.0f)));
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) {     // both forms, selected per value (no branch per value)
            const float a = v[i], a2 = a * a;
            const float small = a * (1.0f + a2 * (-1.0f / 3.0f + a2 * (2.0f / 15.0f)));
            const float big = 1.0f - 2.0f / (1.0f + __expf(2.0f * a));
            v[i] = fabsf(a) < 0.0625f ? small : big;
        }
    }
}

// Curl axes of component c: (curl F)_c = d_{a1} F_{a2} - d_{a2} F_{a1}.
__host__ __device__ constexpr int curl_a1(int c) { return c == 0 ? 1 : (c == 1 ? 2 : 0); }
__host__ __device__ constexpr int curl_a2(int c) { return c == 0 ? 2 : (c == 1 ? 0 : 1); }

// Active components per dimension: 1D {Ez; Hy}, 2D {Ez; Hx, Hy}, 3D all.
__host__ __device__ constexpr bool e_active(int dim, int c) { return dim == 3 || c == 2; }
__host__ __device__ constexpr bool h_active(int dim, int c) { return dim == 3 || (dim == 2 ? c < 2 : c == 1); }
// Axis a carries derivatives in a grid of this dimension.
__host__ __device__ constexpr bool axis_live(int dim, int a) { return a < dim; }

// Device clock: advanced once per step by the tick kernel, read by the others.
struct Clock {
    long long step;                  // index n of the step in progress
    long long next;                  // index of the next step
    double amp[kMaxSources];         // J(t_n) of each source
};

struct SourceDev {
    int comp;
    int lo[3], hi[3];
    double omega_c, tau, t0, amplitude;
    double coef;                     // dt / eps_inf at the source cells
    const double *profile;           // box-sized, or null
};

// Source descriptor carried in kernel arguments (uniform, read through scalar loads).
struct SourceArg {
    int comp;
    int lo[3], hi[3];
    double coef;                     // dt / eps_inf at the source cells
    const double *profile;           // box-sized, or null
};

struct EnergyDev {
    int lo[3], hi[3];
    int every;
    double *partial;                 // [block][3] for this monitor
};

// Arguments of the E / material update of one region.
// One region of a grouped launch: several background regions updated by one kernel launch, the
// blocks of region r being [block0, next block0).
struct RegionDesc {
    int lo[3], ext[3];
    int ext12;
    int block0;
    double inv_eps;
    void *psi[3][2];
    // 3D H regions: psi of the z terms only for z < zlo and z >= zhi, stored per row in
    // zw = (zlo - lo[2]) + (lo[2] + ext[2] - zhi) slots; zw = 0: psi per cell of the region
    int zlo, zhi, zw;
    // 3D E launches of Drude regions: the region's material increments V, material box and
    // coefficients (regions of several Drude materials share one launch)
    void *V[3];
    int mlo[3], mext[3];
    const double *coef;
};
constexpr int kMaxGroup = 32;
// region table of a grouped launch: first blocks (unused entries hold INT_MAX, so every entry can
// be read unconditionally), then the regions
struct RegionTable {
    int block0[kMaxGroup];
    RegionDesc d[kMaxGroup];
};

struct EArgs {
    void *E[3];
    const void *H[3];
    int n[3];
    int per[3];                      // 1: periodic axis, 0: values beyond the grid are zero
    int lo[3], ext[3];               // region box
    int ext12;                       // ext[1] * ext[2]
    double dt, inv_eps;
    // CPML (background regions): psi per E component and curl term, coefficient tables per axis
    void *psi[3][2];
    const double *pml_b[3], *pml_c[3];
    // material box and state
    int mlo[3], mext[3];
    long long mcells;
    void *Pcur[3], *Pnew[3];         // bath/Lorentz: two ping-pong levels; Drude: Pcur = V (read/write)
    void *Ycur[3], *Ynew[3];         // bath: [group][mcells] of 4-vectors
    const void *sigma;               // per material cell (storage type), or null
    double sigma0;
    const double *coef;              // FP64 coefficient table of the material
    void *hid[3];                    // learned closure hidden state [mcells] of float4
    const float *cw;                 // learned closure weights (FP32, kClosureParams)
    int nterm;                       // multi-term material: terms, each with its levels [term][mcells] in Pcur / Pnew
    int drude_mask;                  // multi-term material: bit p set when term p is a Drude term
    // bath coordinate storage: 0 the state type, 1 binary16 of Y yscale, 2 bfloat16 of Y yscale (yinv = 1 / yscale)
    int yfmt;
    double yscale, yinv;
    // thermal (bit 0) and anharmonic (bit 1) bath: extension block of the coefficient table after the
    // modes (per mode: noise amplitude per sqrt(sigma), quartic coefficient, share in the P update;
    // head slot 6: P's noise amplitude per sqrt(sigma)); key of the noise generator
    int bext;
    unsigned key0, key1;
    int nb;                          // bath modes of the material (the table pads to 4 per group)
    double cscale[4];                // closure input scales s_E, s_P, s_V and 1 / s_S
    // sources and clock
    const Clock *clock;
    int nsrc;
    SourceArg src[kMaxSources];
    // energy monitors
    int nen;
    EnergyDev en[kMaxEnergy];
    long long block_base;            // first partial slot of this launch
    const RegionTable *rd;           // grouped launch: region table (nrd > 0), else the box above
    int nrd;
    // Bloch pair (generic kernel only): H of the other part; a read of H across the lower end of
    // periodic axis a returns bcos[a] own - bsin[a] other (bsin = -sin phi_a on the real part,
    // +sin phi_a on the imaginary part); bloch = 0: a real grid, Htw unused
    int bloch;
    const void *Htw[3];
    double bcos[3], bsin[3];
};

struct HArgs {
    const void *E[3];
    void *H[3];
    int n[3];
    int per[3];
    int lo[3], ext[3];
    int ext12;
    double dt;
    void *psi[3][2];
    const double *pml_b[3], *pml_c[3];
    const RegionTable *rd;           // grouped launch: region table (nrd > 0)
    int nrd;
    // Bloch pair: E of the other part; a read of E across the upper end of periodic axis a returns
    // bcos[a] own + bsin[a] other (sign convention of EArgs)
    const void *Etw[3];
    double bcos[3], bsin[3];
};

struct DftArgs {
    int axis, npts;
    int lo[3], ext[3], ext12;
    int n[3], per[3];
    const void *E[2];        // tangential E (t1, t2) or null
    const void *H[2];
    double *stage;           // [slot][4][npts]
    int slot;
};

// Bath coefficients passed by value: head = cE, cP, cPm; per mode a_j, b_j + 1, c_j, sa_j, sb_j.
template <int NG>
struct BathCoef {
    double head[3];
    double md[4 * (NG > 0 ? NG : 1)][5];
};

// Coefficient table layout of a bath / Lorentz material (FP64):
//   [0] cE = w0^2 dt^2 / A      [1] cP = (w0^2 dt^2 - 2) / A
//   [2] cPm = (1 - g0 dt/2 - (dt/2) sum k c) / A
//   [3] rho0 = 1 / w0^2 (energy; rho = rho0 / sigma)   [4] w0^2   [5] 1 / A
//   [6] thermal bath: dt^2 sqrt(2 g0 kT w0^2 / dt) / A, P's noise amplitude per sqrt(sigma)   [7] unused
//   then per mode j (stride 8): a_j, b_j + 1, c_j, sa_j, sb_j, w_j^2, unused, unused
//   with sa_j = (dt/2) k_j a_j / A and sb_j = (dt/2) k_j b_j / A;
//   then, for a thermal or anharmonic bath, per mode j (stride kCoefExt): the noise amplitude per
//   sqrt(sigma) dt^2 sqrt(2 g_j kT w0^2 / dt) / den_j, the quartic coefficient lambda_j dt^2 / den_j
//   (den_j = 1 + g_j dt / 2), and the share (dt/2) k_j / A of the mode's extra term in the P update;
//   for a bath stored in 16 bits (scale s) instead, per mode: c_j s, sa_j / s, sb_j / s (the update of
//   the scaled coordinates Y s).
// Drude table: [0] dE = wp^2 dt^2 / (1 + g dt/2)  [1] dV = (1 - g dt/2)/(1 + g dt/2)  [2] rho = 1/wp^2.
constexpr int kCoefHead = 8;
constexpr int kCoefMode = 8;
constexpr int kCoefExt = 3;          // per mode in the extension block of a thermal / anharmonic bath

// Device memory source of a grid, batch or trainer: the process-wide allocator at the object's
// creation (null callbacks: hipMalloc / hipFree).  Blocks are required to be 256-byte aligned.
struct DevAllocator {
    void *(*alloc)(size_t, void *);
    void (*free)(void *, void *);
    void *ctx;
};
DevAllocator current_allocator();
hipError_t dev_alloc(const DevAllocator &a, void **p, size_t bytes);
void dev_free(const DevAllocator &a, void *p);

}  // namespace fdtdb
