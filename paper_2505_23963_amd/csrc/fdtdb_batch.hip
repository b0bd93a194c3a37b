// Batched 1D FDTD-Bath cavities: many independent 1D grids of uneven length in one launch.
//
// Each workgroup owns a segment of one cavity and loads it together with a halo of T+1 cells on
// each side.  The whole per-cell state (E, H, polarization levels, the N_b bath modes of both
// levels, Drude and CPML auxiliaries) is held in registers while the workgroup advances T steps
// on chip, exchanging neighbour E / H values through LDS with two barriers per step.  Invalid
// data enters from the segment edges at one cell per step and never reaches the owned cells,
// so workgroups never wait on each other; after T steps the owned cells are written back and the
// next launch (graph-captured) continues.  The update arithmetic is the same as the grid path:
// FP64 registers, FP32 or FP64 storage, the three-level Lorentz-Bath recurrences.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fdtdb.h"
#include "fdtdb_internal.h"

namespace fdtdb {
namespace batch {

enum CellType : unsigned char { C_VAC = 0, C_DRUDE = 1, C_BATH = 2, C_PML = 3 };
constexpr int kMaxNG = 8;               // up to 32 bath modes per cell in the on-chip kernel
constexpr int kCavHead = 8;             // per-cavity table head
// per-cavity coefficient table (FP64), stride cav_stride:
//   [0] cE*sigma  [1] cP  [2] cPm  [3] rho (=1/(sigma w0^2))  [4] w0^2  [5] dE (Drude)  [6] dV  [7] rho_drude
//   then per mode j: a_j, b_j + 1, c_j, sa_j, sb_j, w_j^2  (stride 6)
constexpr int kModeStride = 6;

struct Cav {
    int L, off;                         // cells, offset into the global cell arrays
    int src_x, nsrc_steps;              // source cell (-1: none), length of the J table
    int dft_x;                          // DFT cell (-1: none)
    int en_lo, en_hi, en_every;         // energy box [lo, hi) (en_every 0: none)
    double inv_eps[4];                  // 1/eps_inf per cell type
    double src_coef;                    // dt / eps at the source cell
};

struct Seg {
    int cav, x0, own;                   // owned cells [x0, x0 + own)
};

struct Args {
    const Cav *cav;
    const Seg *seg;
    const unsigned char *type;          // per global cell
    const double *pml;                  // per global cell: bE, cE, bH, cH
    const double *coef;                 // per cavity, stride cav_stride
    int cav_stride;
    const double *jtab;                 // per cavity, stride jstride: J(t_n) for n < nsrc_steps
    int jstride;
    void *E, *H, *P0, *P1, *V, *psiE, *psiH;   // per global cell (P0 / P1 ping-pong by step parity)
    void *Y0, *Y1;                      // [group][ncells] of 4-vectors, ping-pong
    int ncells;
    double dt;
    // DFT: per cavity, [2 fields][nf] complex accumulators; frequencies shared
    const double *omega;
    int nf;
    double2 *dft_acc;
    // energy: per cavity, per segment slot, per sample: 3 doubles
    double *en_part;
    int en_cap, seg_slots;
    const int *seg_slot;                // per segment: its slot index inside its cavity
    long long *clock;                   // index of the next step (advanced by k_batch_tick)
    int poison;                         // check mode: every LDS word starts as NaN (FDTDB_POISON_LDS=1 at creation)
};

template <typename T>
using v4 = typename std::conditional<std::is_same<T, float>::value, float4, double4>::type;

__device__ __forceinline__ double wsum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Register-pressure fences (empty asm, no instructions).  fence_ptr makes the coefficient pointer
// opaque at each step so the per-mode coefficients are re-read through the scalar cache instead of
// being hoisted into vector registers.  fence_v4 / fence_d, placed in order before each group of
// four modes, make that group's stored levels (and the running sums) "produced" there, so the
// FP64 conversions of one group are live at a time instead of all 2 x N_b of them.
// coefficient tables are read through the constant address space (scalar loads)
typedef const __attribute__((address_space(4))) double *cdptr;
__device__ __forceinline__ void fence_ptr(cdptr &p) { asm volatile("" : "+s"(p)); }
__device__ __forceinline__ void fence_d(double &v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void fence_v4(float4 &v) { asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w)); }
__device__ __forceinline__ void fence_v4(double4 &v) { asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w)); }

template <typename T, int NG, int NT>
__global__ __launch_bounds__(NT) void k_batch1d(const Args a, const int nsteps, const int halo) {
    using V4 = v4<T>;
    const int step0 = (int)*a.clock;
    __shared__ double sE[NT], sH[NT];
    __shared__ double red[3][NT / 64];
    __shared__ double stage[2][256];    // DFT samples of this block's steps: E(x0), mean H
    const Seg sg = a.seg[blockIdx.x];
    const Cav cv = a.cav[sg.cav];
    const int t = threadIdx.x;
    if (a.poison) {   // check mode: a read of an LDS word that no thread of this launch wrote then shows as NaN
        const double nan = __builtin_nan("");
        sE[t] = nan;
        sH[t] = nan;
        for (int i = t; i < 2 * 256; i += NT) stage[i >> 8][i & 255] = nan;
        if (t < 3 * (NT / 64)) red[t / (NT / 64)][t % (NT / 64)] = nan;
        __syncthreads();
    }
    const int x = sg.x0 - halo + t;
    const bool inside = x >= 0 && x < cv.L;
    const bool own = t >= halo && t < halo + sg.own;
    const int gc = cv.off + (inside ? x : 0);
    const int cav = __builtin_amdgcn_readfirstlane(sg.cav);
    const cdptr cf0 = (cdptr)(a.coef + (long long)cav * a.cav_stride);
    const double inv_dt = 1.0 / a.dt, inv_dt2 = inv_dt * inv_dt;
    unsigned char ty = inside ? a.type[gc] : (unsigned char)C_VAC;
    // ---- load the cell state
    double E = 0.0, H = 0.0, Pa = 0.0, Pb = 0.0, Vd = 0.0, pe = 0.0, ph = 0.0;
    double bE = 1.0, cE = 0.0, bH = 1.0, cH = 0.0;
    V4 ya[NG > 0 ? NG : 1], yb[NG > 0 ? NG : 1];
    const int par = step0 & 1;
    const T *Pcur = static_cast<const T *>(par ? a.P1 : a.P0), *Pprev = static_cast<const T *>(par ? a.P0 : a.P1);
    const V4 *Ycur = static_cast<const V4 *>(par ? a.Y1 : a.Y0), *Yprev = static_cast<const V4 *>(par ? a.Y0 : a.Y1);
    if (inside) {
        E = (double)static_cast<const T *>(a.E)[gc];
        H = (double)static_cast<const T *>(a.H)[gc];
        if (ty == C_BATH) {
            Pa = (double)Pcur[gc];
            Pb = (double)Pprev[gc];
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                ya[g] = Ycur[(long long)g * a.ncells + gc];
                yb[g] = Yprev[(long long)g * a.ncells + gc];
            }
        } else if (ty == C_DRUDE) {
            Vd = (double)static_cast<const T *>(a.V)[gc];
        } else if (ty == C_PML) {
            pe = (double)static_cast<const T *>(a.psiE)[gc];
            ph = (double)static_cast<const T *>(a.psiH)[gc];
            bE = a.pml[4 * (long long)gc + 0];
            cE = a.pml[4 * (long long)gc + 1];
            bH = a.pml[4 * (long long)gc + 2];
            cH = a.pml[4 * (long long)gc + 3];
        }
    }
    const double dt = a.dt;
    const double ie = a.cav[cav].inv_eps[ty];   // indexed in global memory (a runtime index into a
                                                 // private copy would live in scratch)
    for (int s = 0; s < nsteps; ++s) {
        const int n = step0 + s;
        cdptr cf = cf0;
        fence_ptr(cf);
        // ---- E phase: D += dt (dH/dx - J); E = (D - P) / eps;  P, bath
        sH[t] = H;
        __syncthreads();
        const double Hm = t > 0 ? sH[t - 1] : 0.0;        // segment edge: wall or invalid halo
        // the previous step's DFT sample of H: the mean over the node and its left neighbour
        if (s > 0 && cv.dft_x >= 0 && x == cv.dft_x && own) stage[1][s - 1] = 0.5 * (Hm + H);
        double Eo = E, En = E;
        double en_f = 0.0, en_p = 0.0, en_b = 0.0;
        const bool sample = cv.en_every > 0 && (n % cv.en_every) == 0;
        if (inside) {
            double t1 = H - Hm;
            if (ty == C_PML) {
                const double psi = bE * pe + cE * t1;
                pe = psi;
                t1 += psi;
            }
            double src = 0.0;
            if (x == cv.src_x && n < cv.nsrc_steps) src = cv.src_coef * a.jtab[(long long)sg.cav * a.jstride + n];
            if (ty == C_BATH) {
                En = Eo + ie * (dt * t1 - (Pa - Pb)) - src;
                double S = 0.0;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    fence_d(S);
                    fence_d(en_b);
                    fence_v4(ya[g]);
                    fence_v4(yb[g]);
                    const double c0[4] = {(double)ya[g].x, (double)ya[g].y, (double)ya[g].z, (double)ya[g].w};
                    const double c1[4] = {(double)yb[g].x, (double)yb[g].y, (double)yb[g].z, (double)yb[g].w};
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const cdptr md = cf + kCavHead + (4 * g + u) * kModeStride;
                        S += md[3] * c0[u] + md[4] * c1[u];
                        if (sample) en_b += (c0[u] - c1[u]) * (c0[u] - c1[u]) * inv_dt2 + md[5] * c0[u] * c1[u];
                    }
                }
                const double Pn = cf[0] * En - cf[1] * Pa - cf[2] * Pb - S;
                const double dP = Pn - Pb;
                if (sample) {
                    const double v = (Pa - Pb) * inv_dt;
                    en_p = 0.5 * cf[3] * (v * v + cf[4] * Pa * Pb);
                }
                fence_ptr(cf);
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    if (g > 0) {
                        fence_v4(ya[g - 1]);
                        fence_v4(yb[g - 1]);
                    }
                    fence_v4(ya[g]);
                    fence_v4(yb[g]);
                    const double c0[4] = {(double)ya[g].x, (double)ya[g].y, (double)ya[g].z, (double)ya[g].w};
                    const double c1[4] = {(double)yb[g].x, (double)yb[g].y, (double)yb[g].z, (double)yb[g].w};
                    double r[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const cdptr md = cf + kCavHead + (4 * g + u) * kModeStride;
                        r[u] = md[0] * c0[u] + md[1] * c1[u] + md[2] * dP;
                    }
                    // rotate levels: the new level replaces the oldest, rounded to the storage type
                    yb[g] = ya[g];
                    ya[g].x = (T)r[0]; ya[g].y = (T)r[1]; ya[g].z = (T)r[2]; ya[g].w = (T)r[3];
                }
                if (sample) en_b *= 0.5 * cf[3];
                Pb = Pa;
                Pa = (double)(T)Pn;
            } else if (ty == C_DRUDE) {
                En = Eo + ie * (dt * t1 - Vd) - src;
                if (sample) {
                    const double v = Vd * inv_dt;
                    en_p = 0.5 * cf[7] * v * v;
                }
                Vd = (double)(T)(cf[5] * En + cf[6] * Vd);
            } else {
                En = Eo + ie * (dt * t1) - src;
            }
            En = (double)(T)En;
            pe = (double)(T)pe;
            if (sample) en_f = 0.5 / ie * Eo * En + 0.5 * H * H;
        }
        E = En;
        if (sample) {
            // energy of owned cells inside the box: block sum into this segment's slot
            const bool in = own && inside && x >= cv.en_lo && x < cv.en_hi;
            double f0 = in ? en_f : 0.0, f1 = in ? en_p : 0.0, f2 = in ? en_b : 0.0;
            f0 = wsum(f0); f1 = wsum(f1); f2 = wsum(f2);
            if ((t & 63) == 0) { red[0][t >> 6] = f0; red[1][t >> 6] = f1; red[2][t >> 6] = f2; }
            __syncthreads();
            if (t == 0) {
                double s0 = 0.0, s1 = 0.0, s2 = 0.0;
                for (int w = 0; w < NT / 64; ++w) { s0 += red[0][w]; s1 += red[1][w]; s2 += red[2][w]; }
                const int sidx = n / cv.en_every;
                if (sidx < a.en_cap) {
                    double *o = a.en_part + (((long long)sg.cav * a.seg_slots + a.seg_slot[blockIdx.x]) * a.en_cap + sidx) * 3;
                    o[0] = s0; o[1] = s1; o[2] = s2;
                }
            }
        }
        // ---- H phase: H += dt dE/dx (1D, H_y with the curl-law sign)
        sE[t] = E;
        __syncthreads();
        const double Ep = t < NT - 1 ? sE[t + 1] : 0.0;
        if (inside) {
            const double Enb = x + 1 < cv.L ? Ep : 0.0;
            double t2 = Enb - E;
            if (ty == C_PML) {
                const double psi = bH * ph + cH * t2;
                ph = (double)(T)psi;
                t2 += psi;
            }
            H = (double)(T)(H + dt * t2);
        }
        // ---- DFT sample of E at the monitor node (H is sampled at the start of the next step)
        if (cv.dft_x >= 0 && x == cv.dft_x && own) stage[0][s] = E;
    }
    // the last step's H sample, then every sample is visible to the block
    sH[t] = H;
    __syncthreads();
    if (cv.dft_x >= 0 && x == cv.dft_x && own) stage[1][nsteps - 1] = 0.5 * ((t > 0 ? sH[t - 1] : 0.0) + H);
    __syncthreads();
    // ---- write the owned cells back
    if (inside && own) {
        T *Eo = static_cast<T *>(a.E), *Ho = static_cast<T *>(a.H);
        Eo[gc] = (T)E;
        Ho[gc] = (T)H;
        const int pe_ = (step0 + nsteps) & 1;
        T *Pc = static_cast<T *>(pe_ ? a.P1 : a.P0), *Pp = static_cast<T *>(pe_ ? a.P0 : a.P1);
        V4 *Yc = static_cast<V4 *>(pe_ ? a.Y1 : a.Y0), *Yp = static_cast<V4 *>(pe_ ? a.Y0 : a.Y1);
        if (ty == C_BATH) {
            Pc[gc] = (T)Pa;
            Pp[gc] = (T)Pb;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                Yc[(long long)g * a.ncells + gc] = ya[g];
                Yp[(long long)g * a.ncells + gc] = yb[g];
            }
        } else if (ty == C_DRUDE) {
            static_cast<T *>(a.V)[gc] = (T)Vd;
        } else if (ty == C_PML) {
            static_cast<T *>(a.psiE)[gc] = (T)pe;
            static_cast<T *>(a.psiH)[gc] = (T)ph;
        }
    }
    // ---- DFT accumulation for this block's steps (the segment that owns the monitor node)
    const bool owner = cv.dft_x >= sg.x0 && cv.dft_x < sg.x0 + sg.own;
    if (owner) {
        for (int f = t; f < a.nf; f += NT) {
            const double w = a.omega[f];
            double eR = 0.0, eI = 0.0, hR = 0.0, hI = 0.0;
            for (int s = 0; s < nsteps; ++s) {
                double sn, cs;
                sincos(w * (((double)(step0 + s) + 0.5) * dt), &sn, &cs);
                eR += stage[0][s] * (dt * cs);
                eI += stage[0][s] * (dt * sn);
                sincos(w * (((double)(step0 + s) + 1.0) * dt), &sn, &cs);
                hR += stage[1][s] * (dt * cs);
                hI += stage[1][s] * (dt * sn);
            }
            double2 *acc = a.dft_acc + (long long)sg.cav * 2 * a.nf;
            acc[f].x += eR;
            acc[f].y += eI;
            acc[a.nf + f].x += hR;
            acc[a.nf + f].y += hI;
        }
    }
}

// advance the step counter after a launch of nsteps steps
__global__ void k_batch_tick(long long *clock, int nsteps) {
    if (threadIdx.x == 0) clock[0] += nsteps;
}

__global__ void k_jtab(double *jtab, int jstride, const double *par, int ncav, double dt) {
    // par per cavity: omega_c, tau, t0, amplitude, nsteps
    const int c = blockIdx.x;
    if (c >= ncav) return;
    const double wc = par[5 * c], tau = par[5 * c + 1], t0 = par[5 * c + 2], A = par[5 * c + 3];
    const int ns = (int)par[5 * c + 4];
    for (int n = threadIdx.x; n < ns; n += blockDim.x) {
        const double tn = (double)n * dt;
        double J = 0.0;
        if (!(tn > 2.0 * t0)) {
            const double u = tn - t0;
            J = A * exp(-u * u / (2.0 * tau * tau)) * cos(wc * u);
        }
        jtab[(long long)c * jstride + n] = J;
    }
}

// energy read-out: sum the segment slots of one cavity
__global__ void k_batch_energy(const double *part, int seg_slots, int cap, int cav, int nsamp, double *out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsamp) return;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int k = 0; k < seg_slots; ++k) {
        const double *p = part + (((long long)cav * seg_slots + k) * cap + s) * 3;
        a0 += p[0]; a1 += p[1]; a2 += p[2];
    }
    out[3 * s] = a0; out[3 * s + 1] = a1; out[3 * s + 2] = a2;
}

// flux[f] = Re(E conj(H)) with the 1D sign convention: Phi = -Re(E_z conj(H_y))
__global__ void k_batch_flux(const double2 *acc, int nf, int cav, double *flux) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const double2 e = acc[(long long)cav * 2 * nf + f], h = acc[(long long)cav * 2 * nf + nf + f];
    flux[f] = -(e.x * h.x + e.y * h.y);
}

template <typename T, int NG, int NT>
static hipError_t launch_t(const Args &a, int nseg, int nsteps, int halo, hipStream_t s) {
    hipLaunchKernelGGL((k_batch1d<T, NG, NT>), dim3(nseg), dim3(NT), 0, s, a, nsteps, halo);
    hipLaunchKernelGGL(k_batch_tick, dim3(1), dim3(64), 0, s, a.clock, nsteps);
    return hipGetLastError();
}

// Register budget per tile width: 1024 threads hold up to 8 modes per cell, 512 up to 32 (FP32
// storage); FP64 storage runs 256-thread tiles.  Wider tiles are rejected before launch.
static bool tile_fits(bool f64, int nt, int ng) {
    if (f64) return nt == 256;
    if (nt == 1024) return ng <= 2;
    return nt == 256 || nt == 512;
}

template <typename T, int NT>
static hipError_t launch_ng(const Args &a, int ng, int nseg, int nsteps, int halo, hipStream_t s) {
    switch (ng) {
        case 0: return launch_t<T, 0, NT>(a, nseg, nsteps, halo, s);
        case 1: return launch_t<T, 1, NT>(a, nseg, nsteps, halo, s);
        case 2: return launch_t<T, 2, NT>(a, nseg, nsteps, halo, s);
        case 4:
            if constexpr (NT <= 512) return launch_t<T, 4, NT>(a, nseg, nsteps, halo, s);
            return hipErrorInvalidValue;
        case 8:
            if constexpr (NT <= 512) return launch_t<T, 8, NT>(a, nseg, nsteps, halo, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

static hipError_t launch(bool f64, int nt, const Args &a, int ng, int nseg, int nsteps, int halo, hipStream_t s) {
    if (f64) {
        if (nt == 256) return launch_ng<double, 256>(a, ng, nseg, nsteps, halo, s);
        return hipErrorInvalidValue;
    }
    if (nt == 256) return launch_ng<float, 256>(a, ng, nseg, nsteps, halo, s);
    if (nt == 512) return launch_ng<float, 512>(a, ng, nseg, nsteps, halo, s);
    if (nt == 1024) return launch_ng<float, 1024>(a, ng, nseg, nsteps, halo, s);
    return hipErrorInvalidValue;
}

}  // namespace batch
}  // namespace fdtdb

using namespace fdtdb;
using namespace fdtdb::batch;

// Device-resident read-out buffer of fdtdb_batch_energy_noalloc: kNoAllocSamples energy samples of
// three doubles (1.5 MiB), one copy per GPU, held until the process ends.  Host code never uses this
// name as an address: each device's copy is reached through the pointer hipGetSymbolAddress returns,
// taken once per device when the first batch is created on it.
constexpr int kNoAllocSamples = 65536;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[3 * kNoAllocSamples];

// ============================================================================ host runtime
namespace {

thread_local std::string b_err;
std::mutex scratch_mu;
double *scratch_dev[kMaxDevices] = {};     // per device: the address of its `scratch`

fdtdb_status bfail(fdtdb_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    b_err = buf;
    return st;
}

#define BHIP(x)                                                                                 \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) return bfail(FDTDB_E_DEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)
#define BTRY(x)                         \
    do {                                \
        fdtdb_status s_ = (x);          \
        if (s_ != FDTDB_OK) return s_;  \
    } while (0)

struct HostCav {
    int L;
    std::vector<unsigned char> type;
    double eps[4] = {1.0, 1.0, 1.0, 1.0};
    std::vector<double> coef;           // cav_stride doubles
    int nb = 0;
    bool has_bath = false, has_drude = false;
    int src_x = -1;
    double src_par[4] = {0, 0, 0, 0};   // omega_c, width, amplitude, eps
    int dft_x = -1;
    int en_lo = 0, en_hi = 0, en_every = 0;
};

}  // namespace

extern "C" const char *fdtdb_batch_last_error(void) { return b_err.c_str(); }

struct fdtdb_batch_s {
    int dev = 0;                 // the device the batch was created on
    int ncav = 0;
    bool f64 = false;
    double dt = 0.5, R0 = 1e-8;
    int pml = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<HostCav> cavs;
    std::vector<double> omega;          // shared DFT frequencies
    int max_ng = 0;
    bool finalized = false;
    long long steps = 0;
    // tiling
    int steps_per_launch = 0, threads = 0;   // 0: autotune at first step
    // device
    std::vector<void *> allocs;
    Args args{};
    Cav *cav_dev = nullptr;
    Seg *seg_dev = nullptr;
    int *seg_slot_dev = nullptr;
    int nseg = 0, seg_slots = 0, seg_nt = 0, seg_halo = -1;
    std::vector<int> offs;
    int ncells = 0;
    int en_cap = 0;
    int en_slots = 0;            // segment slots per cavity that en_part was sized for
    hipGraphExec_t graph = nullptr;
    int graph_steps = 0;
    std::vector<std::pair<void **, size_t>> state;   // device state arrays and their sizes (autotune scratch)

    DevAllocator mem = current_allocator();
    fdtdb_status alloc(void **p, size_t bytes) {
        if (bytes == 0) bytes = 8;
        hipError_t e = dev_alloc(mem, p, bytes);
        if (e != hipSuccess) return bfail(FDTDB_E_NOMEM, "device allocation of %zu bytes: %s", bytes, hipGetErrorString(e));
        // zeroing on the null stream, asynchronous to the host: finished before the buffer is used on
        // the batch's non-blocking stream
        e = hipMemset(*p, 0, bytes);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) return bfail(FDTDB_E_DEVICE, "hipMemset: %s", hipGetErrorString(e));
        allocs.push_back(*p);
        return FDTDB_OK;
    }
    int cav_stride() const { return kCavHead + kModeStride * 4 * std::max(max_ng, 1); }
};

namespace {

double bpml_sigma(const fdtdb_batch_s *b, int L, double pos) {
    if (b->pml <= 0) return 0.0;
    const double Lp = (double)b->pml;
    const double smax = -4.0 * std::log(b->R0) / (2.0 * Lp);
    double d = 0.0;
    if (pos < Lp) d = Lp - pos;
    else if (pos > (double)(L - 1) - Lp) d = pos - ((double)(L - 1) - Lp);
    if (d <= 0.0) return 0.0;
    const double r = d / Lp;
    return smax * r * r * r;
}

// segment table for a tile shape: own = threads - 2 halo cells per workgroup
fdtdb_status build_segments(fdtdb_batch_s *b, int nt, int halo) {
    const int own = nt - 2 * halo;
    if (own < 1) return bfail(FDTDB_E_INVALID, "tile of %d threads cannot hold a halo of %d", nt, halo);
    std::vector<Seg> segs;
    std::vector<int> slots;
    int max_slots = 0;
    for (int c = 0; c < b->ncav; c++) {
        const HostCav &hc = b->cavs[c];
        int x0 = 0, k = 0;
        while (x0 < hc.L) {
            int w = std::min(own, hc.L - x0);
            // keep the DFT node and its left neighbour in one segment (the H average needs both)
            if (hc.dft_x > x0 && hc.dft_x == x0 + w && w > 1) w -= 1;
            segs.push_back({c, x0, w});
            slots.push_back(k++);
            x0 += w;
        }
        max_slots = std::max(max_slots, k);
    }
    b->nseg = (int)segs.size();
    b->seg_slots = max_slots;
    b->seg_nt = nt;
    b->seg_halo = halo;
    BTRY(b->alloc((void **)&b->seg_dev, sizeof(Seg) * segs.size()));
    BTRY(b->alloc((void **)&b->seg_slot_dev, sizeof(int) * slots.size()));
    BHIP(hipMemcpy(b->seg_dev, segs.data(), sizeof(Seg) * segs.size(), hipMemcpyHostToDevice));
    BHIP(hipMemcpy(b->seg_slot_dev, slots.data(), sizeof(int) * slots.size(), hipMemcpyHostToDevice));
    b->args.seg = b->seg_dev;
    b->args.seg_slot = b->seg_slot_dev;
    b->args.seg_slots = b->seg_slots;
    return FDTDB_OK;
}

fdtdb_status ensure_energy(fdtdb_batch_s *b, long long last_step) {
    int every = 0;
    for (auto &c : b->cavs)
        if (c.en_every) every = every ? std::min(every, c.en_every) : c.en_every;
    if (!every) return FDTDB_OK;
    const long long need = last_step / every + 2;
    // a new tile shape (allowed only before the first step) changes the segment slots per cavity, and
    // with them the buffer's row layout: it is then allocated afresh, zeroed, with nothing to carry over
    const bool reshaped = b->args.en_part && b->en_slots != b->seg_slots;
    if (reshaped && b->steps > 0)
        return bfail(FDTDB_E_STATE, "energy partials laid out for %d segment slots, tiling now has %d", b->en_slots,
                     b->seg_slots);
    if (!reshaped && need <= b->en_cap && b->args.en_part) return FDTDB_OK;
    const int cap = (int)std::max<long long>(need, 2 * (long long)b->en_cap);
    double *nw = nullptr;
    BHIP(hipStreamSynchronize(b->stream));
    BTRY(b->alloc((void **)&nw, 24 * (size_t)b->ncav * b->seg_slots * cap));
    if (b->args.en_part && !reshaped) {
        for (long long r = 0; r < (long long)b->ncav * b->seg_slots; r++)
            BHIP(hipMemcpy(nw + r * cap * 3, b->args.en_part + r * b->en_cap * 3, 24 * (size_t)b->en_cap,
                           hipMemcpyDeviceToDevice));
    }
    b->args.en_part = nw;
    b->en_cap = cap;
    b->en_slots = b->seg_slots;
    b->args.en_cap = cap;
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    return FDTDB_OK;
}

fdtdb_status finalize(fdtdb_batch_s *b) {
    if (b->finalized) return FDTDB_OK;
    // global cell layout
    b->offs.resize(b->ncav);
    int off = 0;
    for (int c = 0; c < b->ncav; c++) { b->offs[c] = off; off += b->cavs[c].L; }
    b->ncells = off;
    const int ng = b->max_ng;
    const size_t w = b->f64 ? 8 : 4;
    Args &a = b->args;
    a.ncells = off;
    a.dt = b->dt;
    BTRY(b->alloc(&a.E, w * off));
    BTRY(b->alloc(&a.H, w * off));
    BTRY(b->alloc(&a.P0, w * off));
    BTRY(b->alloc(&a.P1, w * off));
    BTRY(b->alloc(&a.V, w * off));
    BTRY(b->alloc(&a.psiE, w * off));
    BTRY(b->alloc(&a.psiH, w * off));
    BTRY(b->alloc(&a.Y0, w * 4 * (size_t)std::max(ng, 1) * off));
    BTRY(b->alloc(&a.Y1, w * 4 * (size_t)std::max(ng, 1) * off));
    BTRY(b->alloc((void **)&a.clock, sizeof(long long)));
    std::vector<unsigned char> type(off);
    std::vector<double> pml(4 * (size_t)off);
    const int cs = b->cav_stride();
    std::vector<double> coef((size_t)cs * b->ncav, 0.0);
    std::vector<Cav> cav(b->ncav);
    int jstride = 1;
    std::vector<double> jpar(5 * b->ncav, 0.0);
    for (int c = 0; c < b->ncav; c++) {
        HostCav &hc = b->cavs[c];
        for (int x = 0; x < hc.L; x++) {
            unsigned char ty = hc.type[x];
            const double sE = bpml_sigma(b, hc.L, x), sH = bpml_sigma(b, hc.L, x + 0.5);
            if (ty == C_VAC && (sE > 0.0 || sH > 0.0)) ty = C_PML;
            type[b->offs[c] + x] = ty;
            const double be = std::exp(-sE * b->dt), bh = std::exp(-sH * b->dt);
            double *p = &pml[4 * (size_t)(b->offs[c] + x)];
            p[0] = be; p[1] = be - 1.0; p[2] = bh; p[3] = bh - 1.0;
        }
        std::copy(hc.coef.begin(), hc.coef.end(), coef.begin() + (size_t)c * cs);
        Cav &d = cav[c];
        d.L = hc.L;
        d.off = b->offs[c];
        d.src_x = hc.src_x;
        d.dft_x = hc.dft_x;
        d.en_lo = hc.en_lo;
        d.en_hi = hc.en_hi;
        d.en_every = hc.en_every;
        for (int k = 0; k < 4; k++) d.inv_eps[k] = 1.0 / hc.eps[k];
        d.inv_eps[C_PML] = 1.0;
        d.src_coef = hc.src_x >= 0 ? b->dt / hc.eps[hc.type[hc.src_x]] : 0.0;
        d.nsrc_steps = 0;
        if (hc.src_x >= 0) {
            const double tau = 1.0 / hc.src_par[1], t0 = 5.0 * tau;
            const int ns = (int)std::ceil(2.0 * t0 / b->dt) + 2;
            d.nsrc_steps = ns;
            jstride = std::max(jstride, ns);
            jpar[5 * c] = hc.src_par[0];
            jpar[5 * c + 1] = tau;
            jpar[5 * c + 2] = t0;
            jpar[5 * c + 3] = hc.src_par[2];
            jpar[5 * c + 4] = ns;
        }
    }
    unsigned char *type_dev;
    double *pml_dev, *coef_dev, *jtab, *jpar_dev;
    BTRY(b->alloc((void **)&type_dev, off));
    BTRY(b->alloc((void **)&pml_dev, 8 * pml.size()));
    BTRY(b->alloc((void **)&coef_dev, 8 * coef.size()));
    BTRY(b->alloc((void **)&b->cav_dev, sizeof(Cav) * cav.size()));
    BTRY(b->alloc((void **)&jtab, 8 * (size_t)jstride * b->ncav));
    BTRY(b->alloc((void **)&jpar_dev, 8 * jpar.size()));
    BHIP(hipMemcpy(type_dev, type.data(), off, hipMemcpyHostToDevice));
    BHIP(hipMemcpy(pml_dev, pml.data(), 8 * pml.size(), hipMemcpyHostToDevice));
    BHIP(hipMemcpy(coef_dev, coef.data(), 8 * coef.size(), hipMemcpyHostToDevice));
    BHIP(hipMemcpy(b->cav_dev, cav.data(), sizeof(Cav) * cav.size(), hipMemcpyHostToDevice));
    BHIP(hipMemcpy(jpar_dev, jpar.data(), 8 * jpar.size(), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_jtab, dim3(b->ncav), dim3(64), 0, b->stream, jtab, jstride, jpar_dev, b->ncav, b->dt);
    BHIP(hipGetLastError());
    a.cav = b->cav_dev;
    a.type = type_dev;
    a.pml = pml_dev;
    a.coef = coef_dev;
    a.cav_stride = cs;
    a.jtab = jtab;
    a.jstride = jstride;
    a.nf = (int)b->omega.size();
    double *om;
    BTRY(b->alloc((void **)&om, 8 * std::max<size_t>(1, b->omega.size())));
    if (!b->omega.empty()) BHIP(hipMemcpy(om, b->omega.data(), 8 * b->omega.size(), hipMemcpyHostToDevice));
    a.omega = om;
    BTRY(b->alloc((void **)&a.dft_acc, 32 * (size_t)b->ncav * std::max(a.nf, 1)));
    b->state = {{&a.E, w * off}, {&a.H, w * off}, {&a.P0, w * off}, {&a.P1, w * off}, {&a.V, w * off},
                {&a.psiE, w * off}, {&a.psiH, w * off}, {&a.Y0, w * 4 * (size_t)std::max(ng, 1) * off},
                {&a.Y1, w * 4 * (size_t)std::max(ng, 1) * off}, {(void **)&a.dft_acc, 32 * (size_t)b->ncav * std::max(a.nf, 1)},
                {(void **)&a.clock, sizeof(long long)}};
    BHIP(hipStreamSynchronize(b->stream));
    b->finalized = true;
    return FDTDB_OK;
}

int feasible_threads(const fdtdb_batch_s *b, int nt) { return tile_fits(b->f64, nt, b->max_ng); }

fdtdb_status set_tiling(fdtdb_batch_s *b, int spl, int nt) {
    if (spl < 1 || spl > 254 || !feasible_threads(b, nt)) return bfail(FDTDB_E_INVALID, "unsupported tile %d x %d", spl, nt);
    if (nt - 2 * (spl + 1) < 16) return bfail(FDTDB_E_INVALID, "tile too narrow for %d steps", spl);
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    b->steps_per_launch = spl;
    b->threads = nt;
    return build_segments(b, nt, spl + 1);
}

fdtdb_status enqueue(fdtdb_batch_s *b, int nsteps) {
    BHIP(launch(b->f64, b->threads, b->args, b->max_ng, b->nseg, nsteps, b->seg_halo, b->stream));
    b->steps += nsteps;
    return FDTDB_OK;
}

// Choose the tile shape (steps per launch, threads per workgroup) by timing candidate shapes.
// The timing runs on scratch copies of every state array, with the step counter set far past
// any source pulse; the real state is untouched.
fdtdb_status autotune(fdtdb_batch_s *b) {
    std::vector<void *> real(b->state.size()), scratch(b->state.size());
    for (size_t i = 0; i < b->state.size(); i++) {
        real[i] = *b->state[i].first;
        void *p = nullptr;
        BHIP(dev_alloc(b->mem, &p, b->state[i].second));
        BHIP(hipMemcpyAsync(p, real[i], b->state[i].second, hipMemcpyDeviceToDevice, b->stream));
        scratch[i] = p;
        *b->state[i].first = p;
    }
    const long long far = 1LL << 20;
    BHIP(hipMemcpyAsync(b->args.clock, &far, sizeof far, hipMemcpyHostToDevice, b->stream));
    double *en_saved = b->args.en_part;
    b->args.en_part = nullptr;
    const int cap_saved = b->args.en_cap;
    b->args.en_cap = 0;                 // sample writes are skipped while tuning
    fdtdb_status st = FDTDB_OK;
    int bs = 32, bt = b->f64 ? 256 : 512;
    {
        static const int shapes[][2] = {{16, 256}, {32, 256}, {32, 512}, {64, 512}, {32, 1024}, {64, 1024}, {96, 1024}};
        double best = 1e30;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = bfail(FDTDB_E_DEVICE, "events");
        const long long saved = b->steps;
        for (auto &sh : shapes) {
            if (st != FDTDB_OK) break;
            if (!feasible_threads(b, sh[1]) || sh[1] - 2 * (sh[0] + 1) < 16) continue;
            st = set_tiling(b, sh[0], sh[1]);
            if (st == FDTDB_OK) st = enqueue(b, sh[0]);
            const int reps = std::max(1, 128 / sh[0]);
            if (st == FDTDB_OK && hipEventRecord(e0, b->stream) != hipSuccess) st = bfail(FDTDB_E_DEVICE, "event");
            for (int r = 0; r < reps && st == FDTDB_OK; r++) st = enqueue(b, sh[0]);
            if (st == FDTDB_OK && (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                st = bfail(FDTDB_E_DEVICE, "event");
            float ms = 0.f;
            if (st == FDTDB_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = bfail(FDTDB_E_DEVICE, "event");
            const double per_step = ms / (reps * sh[0]);
            if (st == FDTDB_OK && per_step < best) { best = per_step; bs = sh[0]; bt = sh[1]; }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        b->steps = saved;
    }
    (void)hipStreamSynchronize(b->stream);
    for (size_t i = 0; i < b->state.size(); i++) {
        *b->state[i].first = real[i];
        dev_free(b->mem, scratch[i]);
    }
    b->args.en_part = en_saved;
    b->args.en_cap = cap_saved;
    if (st != FDTDB_OK) return st;
    return set_tiling(b, bs, bt);
}

}  // namespace

// ============================================================================ C ABI
extern "C" {

fdtdb_status fdtdb_batch_create(int ncav, const int64_t *lengths, fdtdb_dtype dtype, double courant, int pml_cells,
                                double pml_R0, void *hip_stream, fdtdb_batch *out) {
    if (!out || !lengths || ncav < 1 || ncav > (1 << 20)) return bfail(FDTDB_E_INVALID, "bad arguments");
    *out = nullptr;
    if (!(courant > 0.0) || courant > 1.0) return bfail(FDTDB_E_UNSTABLE, "courant must be in (0, 1] in 1D");
    if (dtype != FDTDB_F32 && dtype != FDTDB_F64) return bfail(FDTDB_E_INVALID, "bad dtype");
    long long total = 0;
    for (int c = 0; c < ncav; c++) {
        if (lengths[c] < 1 || lengths[c] > (1 << 24)) return bfail(FDTDB_E_INVALID, "bad length of cavity %d", c);
        if (pml_cells > 0 && 2 * pml_cells >= lengths[c]) return bfail(FDTDB_E_INVALID, "CPML too thick for cavity %d", c);
        total += lengths[c];
    }
    if (total >= (1LL << 30)) return bfail(FDTDB_E_INVALID, "too many cells");
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) return bfail(FDTDB_E_DEVICE, "no HIP device");
    if (dev < 0 || dev >= kMaxDevices) return bfail(FDTDB_E_DEVICE, "device %d beyond the supported %d", dev, kMaxDevices);
    {   // once per device, with that device current: the address of its copy of the read-out buffer
        std::lock_guard<std::mutex> lk(scratch_mu);
        if (!scratch_dev[dev]) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return bfail(FDTDB_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            scratch_dev[dev] = static_cast<double *>(ptr);
        }
    }
    auto *b = new fdtdb_batch_s();
    b->dev = dev;
    b->ncav = ncav;
    b->f64 = dtype == FDTDB_F64;
    b->dt = courant;
    b->pml = std::max(0, pml_cells);
    b->R0 = pml_R0 > 0 ? pml_R0 : 1e-8;
    b->cavs.resize(ncav);
    for (int c = 0; c < ncav; c++) {
        b->cavs[c].L = (int)lengths[c];
        b->cavs[c].type.assign(lengths[c], C_VAC);
    }
    // check mode for tests: LDS filled with NaN at the start of every launch
    const char *pz = std::getenv("FDTDB_POISON_LDS");
    b->args.poison = pz && pz[0] == '1';
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return bfail(FDTDB_E_DEVICE, "stream creation failed");
        }
        b->own_stream = true;
    }
    *out = b;
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_destroy(fdtdb_batch b) {
    if (!b) return FDTDB_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    for (void *p : b->allocs) dev_free(b->mem, p);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return FDTDB_OK;
}

static fdtdb_status check_range(fdtdb_batch b, int cav, int64_t lo, int64_t hi) {
    if (!b) return bfail(FDTDB_E_INVALID, "null batch");
    if (b->finalized) return bfail(FDTDB_E_STATE, "batch already stepped");
    if (cav < 0 || cav >= b->ncav) return bfail(FDTDB_E_INVALID, "bad cavity");
    const HostCav &hc = b->cavs[cav];
    if (lo < 0 || hi > hc.L || lo >= hi) return bfail(FDTDB_E_INVALID, "bad range");
    if (b->pml > 0 && (lo < b->pml || hi > hc.L - b->pml)) return bfail(FDTDB_E_INVALID, "material inside the CPML");
    for (int64_t x = lo; x < hi; x++)
        if (hc.type[x] != C_VAC) return bfail(FDTDB_E_INVALID, "materials overlap");
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_set_drude(fdtdb_batch b, int cav, int64_t lo, int64_t hi, double omega_p, double gamma,
                                   double eps_inf) {
    BTRY(check_range(b, cav, lo, hi));
    HostCav &hc = b->cavs[cav];
    if (hc.has_drude && (hc.eps[C_DRUDE] != eps_inf)) return bfail(FDTDB_E_INVALID, "one Drude medium per cavity");
    if (!(eps_inf > 0.0) || !(omega_p >= 0.0) || !(gamma >= 0.0)) return bfail(FDTDB_E_INVALID, "bad Drude parameters");
    const double dt = b->dt;
    if (eps_inf * 4.0 / (dt * dt) - omega_p * omega_p - 4.0 < 0.0) return bfail(FDTDB_E_UNSTABLE, "Drude medium unstable");
    for (int64_t x = lo; x < hi; x++) hc.type[x] = C_DRUDE;
    hc.eps[C_DRUDE] = eps_inf;
    hc.has_drude = true;
    if (hc.coef.empty()) hc.coef.assign(b->cav_stride(), 0.0);
    const double gg = 0.5 * gamma * dt;
    hc.coef[5] = omega_p * omega_p * dt * dt / (1.0 + gg);
    hc.coef[6] = (1.0 - gg) / (1.0 + gg);
    hc.coef[7] = omega_p > 0 ? 1.0 / (omega_p * omega_p) : 0.0;
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_set_lorentz_bath(fdtdb_batch b, int cav, int64_t lo, int64_t hi, double omega0,
                                          double gamma0, double eps_inf, double sigma, int n_bath,
                                          const double *omega_j, const double *gamma_j, const double *k_j) {
    BTRY(check_range(b, cav, lo, hi));
    HostCav &hc = b->cavs[cav];
    if (hc.has_bath) return bfail(FDTDB_E_INVALID, "one Lorentz-Bath medium per cavity");
    if (!(eps_inf > 0.0) || !(omega0 > 0.0) || !(gamma0 >= 0.0) || !(sigma > 0.0) || n_bath < 0 || n_bath > 4 * kMaxNG)
        return bfail(FDTDB_E_INVALID, "bad Lorentz-Bath parameters (n_bath <= %d)", 4 * kMaxNG);
    const double dt = b->dt, w02 = omega0 * omega0;
    if (omega0 * dt >= 2.0 ||
        eps_inf * (4.0 / (dt * dt) - w02) - w02 * sigma - 4.0 * (1.0 - w02 * dt * dt / 4.0) < 0.0)
        return bfail(FDTDB_E_UNSTABLE, "Lorentz medium violates the lattice stability bound");
    for (int j = 0; j < n_bath; j++)
        if (!(omega_j[j] > 0.0) || omega_j[j] * dt >= 2.0 || !(gamma_j[j] >= 0.0))
            return bfail(FDTDB_E_UNSTABLE, "bath mode %d out of range", j);
    int ng = (n_bath + 3) / 4;
    static const int sup[] = {0, 1, 2, 4, 8};
    for (int s : sup)
        if (s >= ng) { ng = s; break; }
    if (ng > b->max_ng) {
        // widen every cavity table to the new mode count
        const int old = b->cav_stride();
        b->max_ng = ng;
        for (auto &c : b->cavs)
            if (!c.coef.empty()) {
                std::vector<double> n2(b->cav_stride(), 0.0);
                std::copy(c.coef.begin(), c.coef.begin() + std::min<int>(old, (int)c.coef.size()), n2.begin());
                c.coef.swap(n2);
            }
    }
    if (hc.coef.empty()) hc.coef.assign(b->cav_stride(), 0.0);
    hc.coef.resize(b->cav_stride(), 0.0);
    for (int64_t x = lo; x < hi; x++) hc.type[x] = C_BATH;
    hc.eps[C_BATH] = eps_inf;
    hc.has_bath = true;
    hc.nb = n_bath;
    double skc = 0.0;
    std::vector<double> aj(n_bath), bj(n_bath), cj(n_bath);
    for (int j = 0; j < n_bath; j++) {
        const double den = 1.0 + 0.5 * gamma_j[j] * dt;
        aj[j] = (2.0 - omega_j[j] * omega_j[j] * dt * dt) / den;
        bj[j] = -2.0 / den;
        cj[j] = k_j[j] * dt / (2.0 * den);
        skc += k_j[j] * cj[j];
    }
    const double A = 1.0 + 0.5 * gamma0 * dt + 0.5 * dt * skc;
    hc.coef[0] = w02 * dt * dt / A * sigma;
    hc.coef[1] = (w02 * dt * dt - 2.0) / A;
    hc.coef[2] = (1.0 - 0.5 * gamma0 * dt - 0.5 * dt * skc) / A;
    hc.coef[3] = 1.0 / (sigma * w02);
    hc.coef[4] = w02;
    for (int j = 0; j < n_bath; j++) {
        double *md = &hc.coef[kCavHead + j * kModeStride];
        md[0] = aj[j];
        md[1] = bj[j] + 1.0;
        md[2] = cj[j];
        md[3] = 0.5 * dt * k_j[j] * aj[j] / A;
        md[4] = 0.5 * dt * k_j[j] * bj[j] / A;
        md[5] = omega_j[j] * omega_j[j];
    }
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_add_source(fdtdb_batch b, int cav, int64_t x, double omega_c, double width, double amplitude) {
    if (!b || b->finalized || cav < 0 || cav >= b->ncav) return bfail(FDTDB_E_INVALID, "bad source call");
    HostCav &hc = b->cavs[cav];
    if (x < 0 || x >= hc.L || hc.src_x >= 0 || !(width > 0.0)) return bfail(FDTDB_E_INVALID, "one source per cavity");
    hc.src_x = (int)x;
    hc.src_par[0] = omega_c;
    hc.src_par[1] = width;
    hc.src_par[2] = amplitude;
    hc.src_par[3] = hc.eps[hc.type[x] == C_VAC ? C_VAC : hc.type[x]];
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_add_dft_flux(fdtdb_batch b, int cav, int64_t x, int nfreq, const double *omega) {
    if (!b || b->finalized || cav < 0 || cav >= b->ncav || nfreq < 1 || nfreq > 4096 || !omega)
        return bfail(FDTDB_E_INVALID, "bad DFT call");
    HostCav &hc = b->cavs[cav];
    if (x < 1 || x >= hc.L || hc.dft_x >= 0) return bfail(FDTDB_E_INVALID, "one DFT point per cavity, 1 <= x < L");
    if (b->omega.empty()) b->omega.assign(omega, omega + nfreq);
    else if ((int)b->omega.size() != nfreq || !std::equal(omega, omega + nfreq, b->omega.begin()))
        return bfail(FDTDB_E_INVALID, "all cavities share one frequency list");
    hc.dft_x = (int)x;
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_add_energy_monitor(fdtdb_batch b, int cav, int64_t lo, int64_t hi, int every) {
    if (!b || b->finalized || cav < 0 || cav >= b->ncav || every < 1) return bfail(FDTDB_E_INVALID, "bad energy call");
    HostCav &hc = b->cavs[cav];
    if (lo < 0 || hi > hc.L || lo >= hi || hc.en_every) return bfail(FDTDB_E_INVALID, "one energy box per cavity");
    hc.en_lo = (int)lo;
    hc.en_hi = (int)hi;
    hc.en_every = every;
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_set_tiling(fdtdb_batch b, int steps_per_launch, int threads_per_block) {
    if (!b) return bfail(FDTDB_E_INVALID, "null batch");
    if (b->steps > 0) return bfail(FDTDB_E_STATE, "the tile shape is fixed once stepping has started");
    BTRY(finalize(b));
    if (steps_per_launch == 0) return autotune(b);
    return set_tiling(b, steps_per_launch, threads_per_block);
}

fdtdb_status fdtdb_batch_get_tiling(fdtdb_batch b, int *steps_per_launch, int *threads_per_block) {
    if (!b || !steps_per_launch || !threads_per_block) return bfail(FDTDB_E_INVALID, "null argument");
    *steps_per_launch = b->steps_per_launch;
    *threads_per_block = b->threads;
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_step(fdtdb_batch b, int64_t nsteps) {
    if (!b || nsteps < 0) return bfail(FDTDB_E_INVALID, "bad step call");
    BTRY(finalize(b));
    if (!b->steps_per_launch) BTRY(autotune(b));
    BTRY(ensure_energy(b, b->steps + nsteps));
    const int spl = b->steps_per_launch;
    int64_t left = nsteps;
    // whole chunks of 16 launches replay one captured graph (the kernels read the device step counter)
    const int chunk = 16 * spl;
    if (left >= chunk && (!b->graph || b->graph_steps != chunk)) {
        if (b->graph) (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
        hipGraph_t graph;
        BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        const long long s0 = b->steps;
        fdtdb_status st = FDTDB_OK;
        for (int k = 0; k < 16 && st == FDTDB_OK; k++) st = enqueue(b, spl);
        hipError_t ce = hipStreamEndCapture(b->stream, &graph);
        b->steps = s0;
        if (st != FDTDB_OK) return st;
        if (ce != hipSuccess) return bfail(FDTDB_E_DEVICE, "capture: %s", hipGetErrorString(ce));
        BHIP(hipGraphInstantiate(&b->graph, graph, nullptr, nullptr, 0));
        (void)hipGraphDestroy(graph);
        b->graph_steps = chunk;
    }
    while (left >= chunk) {
        BHIP(hipGraphLaunch(b->graph, b->stream));
        b->steps += chunk;
        left -= chunk;
    }
    while (left > 0) {
        const int n = (int)std::min<int64_t>(left, spl);
        BTRY(enqueue(b, n));
        left -= n;
    }
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_synchronize(fdtdb_batch b) {
    if (!b) return bfail(FDTDB_E_INVALID, "null batch");
    BHIP(hipStreamSynchronize(b->stream));
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_get_field(fdtdb_batch b, int cav, int component, double *out) {
    if (!b || cav < 0 || cav >= b->ncav || !out || (component != 2 && component != 4))
        return bfail(FDTDB_E_INVALID, "bad field call (1D cavities carry Ez = 2 and Hy = 4)");
    BTRY(finalize(b));
    BHIP(hipStreamSynchronize(b->stream));
    const int L = b->cavs[cav].L, off = b->offs[cav];
    const void *src = component == 2 ? b->args.E : b->args.H;
    if (b->f64) {
        BHIP(hipMemcpy(out, static_cast<const double *>(src) + off, 8 * (size_t)L, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(L);
        BHIP(hipMemcpy(tmp.data(), static_cast<const float *>(src) + off, 4 * (size_t)L, hipMemcpyDeviceToHost));
        for (int i = 0; i < L; i++) out[i] = tmp[i];
    }
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_dft_flux(fdtdb_batch b, int cav, double *flux) {
    if (!b || cav < 0 || cav >= b->ncav || !flux || b->cavs[cav].dft_x < 0) return bfail(FDTDB_E_INVALID, "no DFT point");
    BTRY(finalize(b));
    double *d;
    const int nf = (int)b->omega.size();
    BHIP(dev_alloc(b->mem, (void **)&d, 8 * (size_t)nf));
    hipLaunchKernelGGL(k_batch_flux, dim3((nf + 255) / 256), dim3(256), 0, b->stream, b->args.dft_acc, nf, cav, d);
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipMemcpy(flux, d, 8 * (size_t)nf, hipMemcpyDeviceToHost);
    dev_free(b->mem, d);
    if (e != hipSuccess) return bfail(FDTDB_E_DEVICE, "flux read-out: %s", hipGetErrorString(e));
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_energy(fdtdb_batch b, int cav, double *out, int64_t capacity, int64_t *n_samples) {
    if (!b || cav < 0 || cav >= b->ncav || !b->cavs[cav].en_every) return bfail(FDTDB_E_INVALID, "no energy monitor");
    const HostCav &hc = b->cavs[cav];
    const long long n = b->steps == 0 ? 0 : (b->steps - 1) / hc.en_every + 1;
    if (n_samples) *n_samples = n;
    const long long m = std::min<long long>(n, capacity);
    if (!out || m <= 0) return FDTDB_OK;
    double *d;
    BHIP(dev_alloc(b->mem, (void **)&d, 24 * (size_t)m));
    hipLaunchKernelGGL(k_batch_energy, dim3((m + 255) / 256), dim3(256), 0, b->stream, b->args.en_part, b->seg_slots,
                       b->en_cap, cav, (int)m, d);
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipMemcpy(out, d, 24 * (size_t)m, hipMemcpyDeviceToHost);
    dev_free(b->mem, d);
    if (e != hipSuccess) return bfail(FDTDB_E_DEVICE, "energy read-out: %s", hipGetErrorString(e));
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_energy_noalloc(fdtdb_batch b, int cav, double *out, int64_t capacity, int64_t *n_samples) {
    if (!b || cav < 0 || cav >= b->ncav || !b->cavs[cav].en_every) return bfail(FDTDB_E_INVALID, "no energy monitor");
    const HostCav &hc = b->cavs[cav];
    const long long n = b->steps == 0 ? 0 : (b->steps - 1) / hc.en_every + 1;
    if (n_samples) *n_samples = n;
    const long long m = std::min<long long>(n, capacity);
    if (!out || m <= 0) return FDTDB_OK;
    if (m > kNoAllocSamples)
        return bfail(FDTDB_E_INVALID, "fdtdb_batch_energy_noalloc reads at most %d samples per call (asked for %lld)",
                     kNoAllocSamples, m);
    double *buf = scratch_dev[b->dev];
    if (!buf) return bfail(FDTDB_E_STATE, "no read-out buffer on device %d", b->dev);
    hipLaunchKernelGGL(k_batch_energy, dim3((m + 255) / 256), dim3(256), 0, b->stream, b->args.en_part, b->seg_slots,
                       b->en_cap, cav, (int)m, buf);
    BHIP(hipGetLastError());
    BHIP(hipStreamSynchronize(b->stream));
    BHIP(hipMemcpy(out, buf, 24 * (size_t)m, hipMemcpyDeviceToHost));
    return FDTDB_OK;
}

fdtdb_status fdtdb_batch_steps_done(fdtdb_batch b, int64_t *steps) {
    if (!b || !steps) return bfail(FDTDB_E_INVALID, "null argument");
    *steps = b->steps;
    return FDTDB_OK;
}

}  // extern "C"
