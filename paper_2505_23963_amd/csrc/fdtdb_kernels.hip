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

// value at coordinate-1 / coordinate+1 along an axis, with the axis boundary rule
template <typename T>
__device__ __forceinline__ double at_minus(const void *f, long long q, int coord, long long stride, int n, int per) {
    if (coord > 0) return ldd<T>(f, q - stride);
    return per ? ldd<T>(f, q + (long long)(n - 1) * stride) : 0.0;
}
template <typename T>
__device__ __forceinline__ double at_plus(const void *f, long long q, int coord, long long stride, int n, int per) {
    if (coord < n - 1) return ldd<T>(f, q + stride);
    return per ? ldd<T>(f, q - (long long)(n - 1) * stride) : 0.0;
}

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

// ---------------------------------------------------------------------------------------------
// E / material update
// ---------------------------------------------------------------------------------------------
template <int DIM, typename T, int KIND, int NG, bool PML, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_update_e(const EArgs a) {
    using V4 = vec4_t<T>;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const bool live = t < a.ext[0] * a.ext12;
    const long long s0 = (long long)a.n[1] * a.n[2], s1 = a.n[2];
    double ef = 0.0, ep = 0.0, eb = 0.0;   // energy densities of this cell (when sampled)
    bool sample = false;
    if (ENERGY) {
        const long long st = a.clock->step;
        for (int e = 0; e < a.nen; ++e) sample |= (st % a.en[e].every) == 0;
    }
    int i = 0, j = 0, k = 0;
    if (live) {
        unflatten<DIM>(t, a.lo, a.ext, a.ext12, i, j, k);
        const long long q = i * s0 + j * s1 + k;
        const int coord[3] = {i, j, k};
        const long long stride[3] = {s0, s1, 1};
        long long m = 0;
        double sig = a.sigma0;
        if (KIND != K_BACKGROUND) {
            m = ((long long)(i - a.mlo[0]) * a.mext[1] + (j - a.mlo[1])) * a.mext[2] + (k - a.mlo[2]);
            if (a.sigma) sig = ldd<T>(a.sigma, m);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (!e_active(DIM, c)) continue;
            const int a1 = curl_a1(c), a2 = curl_a2(c);
            double t1 = 0.0, t2 = 0.0;
            if (axis_live(DIM, a1) && h_active(DIM, a2))
                t1 = ldd<T>(a.H[a2], q) - at_minus<T>(a.H[a2], q, coord[a1], stride[a1], a.n[a1], a.per[a1]);
            if (axis_live(DIM, a2) && h_active(DIM, a1))
                t2 = ldd<T>(a.H[a1], q) - at_minus<T>(a.H[a1], q, coord[a2], stride[a2], a.n[a2], a.per[a2]);
            if (PML) {
                if (a.psi[c][0]) {
                    T *ps = static_cast<T *>(a.psi[c][0]);
                    const long long r = t;
                    const double psi = a.pml_b[a1][coord[a1]] * (double)ps[r] + a.pml_c[a1][coord[a1]] * t1;
                    ps[r] = (T)psi;
                    t1 += psi;
                }
                if (a.psi[c][1]) {
                    T *ps = static_cast<T *>(a.psi[c][1]);
                    const long long r = t;
                    const double psi = a.pml_b[a2][coord[a2]] * (double)ps[r] + a.pml_c[a2][coord[a2]] * t2;
                    ps[r] = (T)psi;
                    t2 += psi;
                }
            }
            const double curl = t1 - t2;
            // soft current sources on this component
            double srcterm = 0.0;
            for (int s = 0; s < a.nsrc; ++s) {
                const SourceDev &S = a.src[s];
                if (S.comp != c) continue;
                if (i < S.lo[0] || i >= S.hi[0] || j < S.lo[1] || j >= S.hi[1] || k < S.lo[2] || k >= S.hi[2]) continue;
                double prof = 1.0;
                if (S.profile) {
                    const long long sl = ((long long)(i - S.lo[0]) * (S.hi[1] - S.lo[1]) + (j - S.lo[1])) * (S.hi[2] - S.lo[2]) + (k - S.lo[2]);
                    prof = S.profile[sl];
                }
                srcterm += S.coef * a.clock->amp[s] * prof;
            }
            T *Ec = static_cast<T *>(a.E[c]);
            const double Eo = (double)Ec[q];
            double En;
            if (KIND == K_BACKGROUND) {
                En = Eo + a.inv_eps * (a.dt * curl) - srcterm;
                if (ENERGY && sample) ef += 0.5 / a.inv_eps * Eo * En;
            } else if (KIND == K_DRUDE) {
                T *Vp = static_cast<T *>(a.Pcur[c]);
                const double V = (double)Vp[m];
                En = Eo + a.inv_eps * (a.dt * curl - V) - srcterm;
                Vp[m] = (T)(a.coef[0] * En + a.coef[1] * V);
                if (ENERGY && sample) {
                    ef += 0.5 / a.inv_eps * Eo * En;
                    const double v = V / a.dt;
                    ep += 0.5 * a.coef[2] * v * v;
                }
            } else {  // K_BATH (NG == 0: plain Lorentz)
                T *Pc_ = static_cast<T *>(a.Pcur[c]);
                T *Pn_ = static_cast<T *>(a.Pnew[c]);
                const double Pc = (double)Pc_[m], Pp = (double)Pn_[m];
                En = Eo + a.inv_eps * (a.dt * curl - (Pc - Pp)) - srcterm;
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
                const double Pnew = cf[0] * sig * En - cf[1] * Pc - cf[2] * Pp - S;
                Pn_[m] = (T)Pnew;
                const double dP = Pnew - Pp;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const double *md = cf + kCoefHead + 4 * g * kCoefMode;
                    V4 o;
                    o.x = (T)(md[0 * kCoefMode + 0] * (double)yc[g].x + md[0 * kCoefMode + 1] * (double)yp[g].x + md[0 * kCoefMode + 2] * dP);
                    o.y = (T)(md[1 * kCoefMode + 0] * (double)yc[g].y + md[1 * kCoefMode + 1] * (double)yp[g].y + md[1 * kCoefMode + 2] * dP);
                    o.z = (T)(md[2 * kCoefMode + 0] * (double)yc[g].z + md[2 * kCoefMode + 1] * (double)yp[g].z + md[2 * kCoefMode + 2] * dP);
                    o.w = (T)(md[3 * kCoefMode + 0] * (double)yc[g].w + md[3 * kCoefMode + 1] * (double)yp[g].w + md[3 * kCoefMode + 2] * dP);
                    Yn[(long long)g * a.mcells + m] = o;
                }
                if (ENERGY && sample) {
                    ef += 0.5 / a.inv_eps * Eo * En;
                    const double rho = cf[3] / sig;
                    const double v = (Pc - Pp) / a.dt;
                    ep += 0.5 * rho * (v * v + cf[4] * Pc * Pp);
                    double bsum = 0.0;
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        const double *md = cf + kCoefHead + 4 * g * kCoefMode;
                        const double c0 = (double)yc[g].x, p0 = (double)yp[g].x;
                        const double c1 = (double)yc[g].y, p1 = (double)yp[g].y;
                        const double c2 = (double)yc[g].z, p2 = (double)yp[g].z;
                        const double c3 = (double)yc[g].w, p3 = (double)yp[g].w;
                        bsum += (c0 - p0) * (c0 - p0) / (a.dt * a.dt) + md[0 * kCoefMode + 5] * c0 * p0;
                        bsum += (c1 - p1) * (c1 - p1) / (a.dt * a.dt) + md[1 * kCoefMode + 5] * c1 * p1;
                        bsum += (c2 - p2) * (c2 - p2) / (a.dt * a.dt) + md[2 * kCoefMode + 5] * c2 * p2;
                        bsum += (c3 - p3) * (c3 - p3) / (a.dt * a.dt) + md[3 * kCoefMode + 5] * c3 * p3;
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
    if (ENERGY && sample) {
        // one partial per monitor per block; cells outside a monitor's box contribute zero
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
}

// ---------------------------------------------------------------------------------------------
// H update
// ---------------------------------------------------------------------------------------------
template <int DIM, typename T, bool PML>
__global__ __launch_bounds__(kBlock) void k_update_h(const HArgs a) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= a.ext[0] * a.ext12) return;
    int i, j, k;
    unflatten<DIM>(t, a.lo, a.ext, a.ext12, i, j, k);
    const long long s0 = (long long)a.n[1] * a.n[2], s1 = a.n[2];
    const long long q = i * s0 + j * s1 + k;
    const int coord[3] = {i, j, k};
    const long long stride[3] = {s0, s1, 1};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (!h_active(DIM, c)) continue;
        const int a1 = curl_a1(c), a2 = curl_a2(c);
        double t1 = 0.0, t2 = 0.0;
        if (axis_live(DIM, a1) && e_active(DIM, a2))
            t1 = at_plus<T>(a.E[a2], q, coord[a1], stride[a1], a.n[a1], a.per[a1]) - ldd<T>(a.E[a2], q);
        if (axis_live(DIM, a2) && e_active(DIM, a1))
            t2 = at_plus<T>(a.E[a1], q, coord[a2], stride[a2], a.n[a2], a.per[a2]) - ldd<T>(a.E[a1], q);
        if (PML) {
            if (a.psi[c][0]) {
                T *ps = static_cast<T *>(a.psi[c][0]);
                const double psi = a.pml_b[a1][coord[a1]] * (double)ps[t] + a.pml_c[a1][coord[a1]] * t1;
                ps[t] = (T)psi;
                t1 += psi;
            }
            if (a.psi[c][1]) {
                T *ps = static_cast<T *>(a.psi[c][1]);
                const double psi = a.pml_b[a2][coord[a2]] * (double)ps[t] + a.pml_c[a2][coord[a2]] * t2;
                ps[t] = (T)psi;
                t2 += psi;
            }
        }
        T *Hc = static_cast<T *>(a.H[c]);
        Hc[q] = (T)((double)Hc[q] - a.dt * (t1 - t2));
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
__global__ __launch_bounds__(kBlock) void k_dft_flush(const double *stage, const double *tw, int npts, int nf,
                                                     int nslots, double2 *acc) {
    __shared__ double2 ltw[kDftSlots][kDftFreqTile];
    const int field = blockIdx.y;
    const int f0 = blockIdx.z * kDftFreqTile;
    const int hsel = field >= 2 ? 2 : 0;
    for (int id = threadIdx.x; id < nslots * kDftFreqTile; id += kBlock) {
        const int b = id / kDftFreqTile, f = id - b * kDftFreqTile;
        double2 v = make_double2(0.0, 0.0);
        if (f0 + f < nf) {
            const double *o = tw + 4 * ((long long)b * nf + f0 + f);
            v = make_double2(o[hsel], o[hsel + 1]);
        }
        ltw[b][f] = v;
    }
    __syncthreads();
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npts) return;
    double re[kDftFreqTile], im[kDftFreqTile];
#pragma unroll
    for (int f = 0; f < kDftFreqTile; ++f) { re[f] = 0.0; im[f] = 0.0; }
    for (int b = 0; b < nslots; ++b) {
        const double x = stage[((long long)b * 4 + field) * npts + p];
#pragma unroll
        for (int f = 0; f < kDftFreqTile; ++f) {
            re[f] += x * ltw[b][f].x;
            im[f] += x * ltw[b][f].y;
        }
    }
#pragma unroll
    for (int f = 0; f < kDftFreqTile; ++f) {
        if (f0 + f >= nf) continue;
        double2 *d = acc + ((long long)field * nf + f0 + f) * npts + p;
        double2 v = *d;
        v.x += re[f];
        v.y += im[f];
        *d = v;
    }
}

// flux[f] = Re sum_p (E1 conj(H2) - E2 conj(H1))
__global__ __launch_bounds__(kBlock) void k_dft_flux(const double2 *acc, int npts, int nf, double *flux) {
    const int f = blockIdx.x;
    const double2 *e1 = acc + (0LL * nf + f) * npts, *e2 = acc + (1LL * nf + f) * npts;
    const double2 *h1 = acc + (2LL * nf + f) * npts, *h2 = acc + (3LL * nf + f) * npts;
    double s = 0.0, z1 = 0.0, z2 = 0.0;
    for (int p = threadIdx.x; p < npts; p += kBlock)
        s += (e1[p].x * h2[p].x + e1[p].y * h2[p].y) - (e2[p].x * h1[p].x + e2[p].y * h1[p].y);
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

// ---------------------------------------------------------------------------------------------
// launchers (host side)
// ---------------------------------------------------------------------------------------------
static inline unsigned nblocks(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <int DIM, typename T, int KIND, int NG, bool PML>
static hipError_t launch_e_pml(const EArgs &a, bool energy, hipStream_t s) {
    const long long n = (long long)a.ext[0] * a.ext12;
    if (n == 0) return hipSuccess;
    if (energy)
        hipLaunchKernelGGL((k_update_e<DIM, T, KIND, NG, PML, true>), dim3(nblocks(n)), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_update_e<DIM, T, KIND, NG, PML, false>), dim3(nblocks(n)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int DIM, typename T>
static hipError_t launch_e_dim(const EArgs &a, int kind, int ng, bool pml, bool energy, hipStream_t s) {
    if (kind == K_BACKGROUND)
        return pml ? launch_e_pml<DIM, T, K_BACKGROUND, 0, true>(a, energy, s)
                   : launch_e_pml<DIM, T, K_BACKGROUND, 0, false>(a, energy, s);
    if (kind == K_DRUDE) return launch_e_pml<DIM, T, K_DRUDE, 0, false>(a, energy, s);
    if (kind == K_BATH) {
        switch (ng) {
            case 0: return launch_e_pml<DIM, T, K_BATH, 0, false>(a, energy, s);
            case 1: return launch_e_pml<DIM, T, K_BATH, 1, false>(a, energy, s);
            case 2: return launch_e_pml<DIM, T, K_BATH, 2, false>(a, energy, s);
            case 3: return launch_e_pml<DIM, T, K_BATH, 3, false>(a, energy, s);
            case 4: return launch_e_pml<DIM, T, K_BATH, 4, false>(a, energy, s);
            case 6: return launch_e_pml<DIM, T, K_BATH, 6, false>(a, energy, s);
            case 8: return launch_e_pml<DIM, T, K_BATH, 8, false>(a, energy, s);
            case 12: return launch_e_pml<DIM, T, K_BATH, 12, false>(a, energy, s);
            case 16: return launch_e_pml<DIM, T, K_BATH, 16, false>(a, energy, s);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_update_e(int dim, bool f64, const EArgs &a, int kind, int ng, bool pml, bool energy,
                           hipStream_t s) {
    if (f64) {
        if (dim == 1) return launch_e_dim<1, double>(a, kind, ng, pml, energy, s);
        if (dim == 2) return launch_e_dim<2, double>(a, kind, ng, pml, energy, s);
        return launch_e_dim<3, double>(a, kind, ng, pml, energy, s);
    }
    if (dim == 1) return launch_e_dim<1, float>(a, kind, ng, pml, energy, s);
    if (dim == 2) return launch_e_dim<2, float>(a, kind, ng, pml, energy, s);
    return launch_e_dim<3, float>(a, kind, ng, pml, energy, s);
}

template <int DIM, typename T>
static hipError_t launch_h_dim(const HArgs &a, bool pml, hipStream_t s) {
    const long long n = (long long)a.ext[0] * a.ext12;
    if (n == 0) return hipSuccess;
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
    hipLaunchKernelGGL(k_dft_flush, dim3(nblocks(npts), 4, (nf + kDftFreqTile - 1) / kDftFreqTile), dim3(kBlock), 0, s,
                       stage, tw, npts, nf, nslots, acc);
    return hipGetLastError();
}

hipError_t launch_dft_flux(const double2 *acc, int npts, int nf, double *flux, hipStream_t s) {
    hipLaunchKernelGGL(k_dft_flux, dim3(nf), dim3(kBlock), 0, s, acc, npts, nf, flux);
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
