"""The five benchmark workloads and their reduced parity variants.

Every random number comes from Philox4x32-10 keyed by (seed, stream id);
streams: 1 couplings, 2 sigma field, 3 cavity lengths, 4 detunings,
5 training windows, 6 source profiles.  Readings of values the workload
statements leave open are fixed here (see the design notes of the repository):

* Drude mirrors: omega_p = 10, gamma = 0.01, eps_inf = 10 (the smallest
  round background above the explicit-scheme stability bound at Courant 0.5).
* "Ohmic" couplings: damping profile Gamma_B(w) = 0.01 exp(-(w - omega0)/1),
  k_j = sqrt(2 dw Gamma_B(w_j) / pi) * (1 + 0.1 xi_j), xi_j ~ N(0,1) clipped
  to +-3 (the uniform-bath rule k_b^2 = 2 dw dephasing / pi applied mode by
  mode), gamma_j = dw / 10.
* Gaussian pulse: soft current, tau = 1/width, t0 = 5 tau, off after 2 t0.
"""
from __future__ import annotations

import numpy as np

from .philox import Stream
from .problem import (CLOSED, PERIODIC, PML, DftFlux, Drude, EnergyMonitor, LorentzBath, Problem,
                      Source, bath_grid, box, freq_grid)

MIRROR = dict(omega_p=10.0, gamma=0.01, eps_inf=10.0)


def ohmic_bath(nb: int, lo: float, hi: float, omega0: float, seed: int, stream: int = 1,
               offset_blocks: int = 0, gamma_b0: float = 0.01, omega_cut: float = 1.0):
    """Bath frequencies, dampings and couplings drawn from the seeded Ohmic recipe."""
    w = bath_grid(nb, lo, hi)
    dw = (hi - lo) / (nb - 1) if nb > 1 else 1.0
    rs = Stream(seed, stream)
    rs.block = offset_blocks
    xi = np.clip(rs.normal(nb), -3.0, 3.0)
    gam_b = gamma_b0 * np.exp(-(w - omega0) / omega_cut)
    k = np.sqrt(2.0 * dw * gam_b / np.pi) * (1.0 + 0.1 * xi)
    g = np.full(nb, dw / 10.0)
    return w, g, k


def gaussian_pulse(comp, bx, profile=None, omega_c=1.0, width=0.5):
    return Source(comp=comp, box=bx, omega_c=omega_c, width=width, amplitude=1.0, profile=profile)


# ----------------------------------------------------------------------------------------------
# 1 - 1D Fabry-Perot, FP64
# ----------------------------------------------------------------------------------------------
def config1_1d(steps: int = 20000, nb: int = 16, nfreq: int = 512, dtype: str = "f64") -> Problem:
    """2048 cells: PML 64 | vac 40 | Drude 20 | LB 1800 | Drude 20 | vac 40 | PML 64."""
    N = 2048
    edges = np.cumsum([0, 64, 40, 20, 1800, 20, 40, 64])
    assert edges[-1] == N
    w, g, k = ohmic_bath(nb, 0.8, 1.2, 1.0, seed=1001)
    p = Problem(name="1d-fabry-perot-f64", ndim=1, n=(N, 1, 1), bc=(PML, PERIODIC, PERIODIC),
                pml_cells=(64, 0, 0), dtype=dtype, steps=steps)
    p.materials += [
        Drude(box((edges[2], edges[3])), **MIRROR),
        LorentzBath(box((edges[3], edges[4])), omega0=1.0, gamma0=0.0, eps_inf=1.0, sigma=0.05,
                    n_bath=nb, omega_j=w, gamma_j=g, k_j=k),
        Drude(box((edges[4], edges[5])), **MIRROR),
    ]
    p.sources.append(gaussian_pulse(2, box((134, 135))))
    om = freq_grid(nfreq)
    p.dfts += [DftFlux(0, box((1914, 1915)), om), DftFlux(0, box((1964, 1965)), om)]
    p.energies.append(EnergyMonitor(box((edges[2], edges[5])), every=10))
    return p


# ----------------------------------------------------------------------------------------------
# 2 - 3D planar cavity, FP32 (the benchmark workload)
# ----------------------------------------------------------------------------------------------
def config2_3d(nx: int = 256, ny: int = 256, steps: int = 5000, nb: int = 8, nfreq: int = 256,
               dtype: str = "f32", seed: int = 1002, sigma_window=None) -> Problem:
    """nx x ny x 512, periodic x,y; z: PML 32 | vac 12 | Drude 12 | LB 400 | Drude 12 | vac 12 | PML 32.

    sigma ~ U[0.01, 0.1] per cell of the LB layer.  The 12-cell Drude mirrors
    at omega_p = 10 are opaque (amplitude transmission ~1e-24), so the plane
    source (z = 66) and the flux plane (z = 446) sit inside the cavity, 10
    cells from the layer edges, as for the 1D cavity.  The field is drawn for the
    full 256 x 256 plane; a crop (nx, ny < 256) takes its corner, or the window
    sigma_window = (x0, y0) of it, so a crop sees the same sigma values as the
    full grid there.
    """
    NZ = 512
    edges = np.cumsum([0, 32, 12, 12, 400, 12, 12, 32])
    assert edges[-1] == NZ
    full = Stream(seed, 2).uniform(256 * 256 * 400, 0.01, 0.1).reshape(256, 256, 400)
    x0, y0 = sigma_window or (0, 0)
    idx_x = (x0 + np.arange(nx)) % 256
    idx_y = (y0 + np.arange(ny)) % 256
    sig = np.ascontiguousarray(full[idx_x][:, idx_y])
    w, g, k = ohmic_bath(nb, 0.8, 1.2, 1.0, seed=seed)
    p = Problem(name="3d-planar-cavity-f32", ndim=3, n=(nx, ny, NZ), bc=(PERIODIC, PERIODIC, PML),
                pml_cells=(0, 0, 32), dtype=dtype, steps=steps)
    full_xy = ((0, nx), (0, ny))
    p.materials += [
        Drude(box(*full_xy, (edges[2], edges[3])), **MIRROR),
        LorentzBath(box(*full_xy, (edges[3], edges[4])), omega0=1.0, gamma0=0.0, eps_inf=1.0,
                    sigma_cells=sig, n_bath=nb, omega_j=w, gamma_j=g, k_j=k),
        Drude(box(*full_xy, (edges[4], edges[5])), **MIRROR),
    ]
    p.sources.append(gaussian_pulse(0, box(*full_xy, (edges[3] + 10, edges[3] + 11))))
    p.dfts.append(DftFlux(2, box(*full_xy, (edges[4] - 10, edges[4] - 9)), freq_grid(nfreq)))
    return p


# ----------------------------------------------------------------------------------------------
# 3 - batched 1D cavities, FP32
# ----------------------------------------------------------------------------------------------
def config3_cavities(ncav: int = 64, steps: int = 50000, nb: int = 32, nfreq: int = 512,
                     dtype: str = "f32", lengths=None, seed: int = 1003):
    """64 independent 1D cavities: PML 32 | vac 8 | Drude 20 | LB L-120 | Drude 20 | vac 8 | PML 32.

    L ~ U[1500, 4000], sigma log-uniform on [1e-3, 1e-1], omega0 = 1 + delta with
    delta ~ U[-0.1, 0.1], N_b modes on omega0 +- 0.2 with Ohmic couplings.
    Returns a list of 1D Problems (one per cavity).
    """
    if lengths is None:
        lengths = Stream(seed, 3).integers(ncav, 1500, 4000)
    lengths = np.asarray(lengths, dtype=np.int64)[:ncav]
    sig = 10.0 ** Stream(seed, 2).uniform(ncav, -3.0, -1.0)
    delta = Stream(seed, 4).uniform(ncav, -0.1, 0.1)
    om = freq_grid(nfreq)
    cavs = []
    for c in range(ncav):
        L = int(lengths[c])
        w0 = 1.0 + float(delta[c])
        w, g, k = ohmic_bath(nb, w0 - 0.2, w0 + 0.2, w0, seed=seed, offset_blocks=64 * c)
        e = np.cumsum([0, 32, 8, 20, L - 120, 20, 8, 32])
        p = Problem(name=f"cavity{c}", ndim=1, n=(L, 1, 1), bc=(PML, PERIODIC, PERIODIC),
                    pml_cells=(32, 0, 0), dtype=dtype, steps=steps)
        p.materials += [
            Drude(box((e[2], e[3])), **MIRROR),
            LorentzBath(box((e[3], e[4])), omega0=w0, gamma0=0.0, eps_inf=1.0, sigma=float(sig[c]),
                        n_bath=nb, omega_j=w, gamma_j=g, k_j=k),
            Drude(box((e[4], e[5])), **MIRROR),
        ]
        p.sources.append(gaussian_pulse(2, box((e[3] + 10, e[3] + 11))))
        p.dfts.append(DftFlux(0, box((e[4] - 10, e[4] - 9)), om))
        p.energies.append(EnergyMonitor(box((e[3], e[4])), every=10))
        cavs.append(p)
    return cavs


# ----------------------------------------------------------------------------------------------
# 4 - 2D TM grid with a Lorentz-Bath patch (explicit N_b = 64, learned-closure target)
# ----------------------------------------------------------------------------------------------
def config4_2d(n: int = 2048, patch=(512, 1536), steps: int = 10000, nb: int = 64, nfreq: int = 256,
               dtype: str = "f32", src_x: int = 48, flux_x: int = 1800) -> Problem:
    """n x n TM grid, PML 32 on all sides, Lorentzian-form bath on the patch."""
    p = Problem(name="2d-tm-patch", ndim=2, n=(n, n, 1), bc=(PML, PML, PERIODIC), pml_cells=(32, 32, 0),
                dtype=dtype, steps=steps)
    p.materials.append(LorentzBath(box(patch, patch), omega0=1.0, gamma0=0.001, eps_inf=1.0, sigma=0.05,
                                   n_bath=nb, form="lorentzian", width=0.4, bath_gamma=0.4 / (nb - 1) / 2,
                                   dephasing=0.02))
    p.sources.append(gaussian_pulse(2, box((src_x, src_x + 1), (32, n - 32))))
    p.dfts.append(DftFlux(0, box((flux_x, flux_x + 1), (32, n - 32)), freq_grid(nfreq)))
    return p


# ----------------------------------------------------------------------------------------------
# 5 - large 3D, FP32 state, FP64 DFT
# ----------------------------------------------------------------------------------------------
def config5_3d_large(nx: int = 512, ny: int = 512, steps: int = 4000, nb: int = 16, nfreq: int = 256,
                     dtype: str = "f32", waist: float = 64.0) -> Problem:
    """nx x ny x 512, periodic x,y; z: PML 32 | vac 121 | LB 205 | vac 122 | PML 32."""
    NZ = 512
    e = np.cumsum([0, 32, 121, 205, 122, 32])
    assert e[-1] == NZ
    w, g, k = ohmic_bath(nb, 0.8, 1.2, 1.0, seed=1005)
    p = Problem(name="3d-large", ndim=3, n=(nx, ny, NZ), bc=(PERIODIC, PERIODIC, PML), pml_cells=(0, 0, 32),
                dtype=dtype, steps=steps)
    xy = ((0, nx), (0, ny))
    p.materials.append(LorentzBath(box(*xy, (e[2], e[3])), omega0=1.0, gamma0=0.0, eps_inf=1.0, sigma=0.05,
                                   n_bath=nb, omega_j=w, gamma_j=g, k_j=k))
    X, Y = np.meshgrid(np.arange(nx) - nx / 2 + 0.5, np.arange(ny) - ny / 2 + 0.5, indexing="ij")
    prof = np.exp(-(X ** 2 + Y ** 2) / waist ** 2).reshape(nx, ny, 1)
    p.sources.append(gaussian_pulse(0, box(*xy, (42, 43)), profile=prof))
    p.dfts.append(DftFlux(2, box(*xy, (470, 471)), freq_grid(nfreq)))
    return p


def thermal_setup(p: Problem, kT: float = 1e-6, lam: float = 50.0, seed: int = 0x2505_23963) -> Problem:
    """The large 3D layout with its Lorentz-Bath slab made thermal (temperature kT, noise seed) and
    anharmonic (quartic coefficient lam on every mode): the thermal / anharmonic benchmark line."""
    m = p.materials[0]
    m.kT, m.noise_seed, m.anharmonic = kT, seed, np.full(m.n_bath, lam)
    return p


# ----------------------------------------------------------------------------------------------
# learned closure: seeded initial weights (stream 5)
# ----------------------------------------------------------------------------------------------
CLOSURE_SHAPES = (("W1", (32, 7)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)), ("W3", (5, 32)), ("b3", (5,)))


def closure_init(seed: int, hidden_scale: float = 0.3, state_scale: float = 0.0, force_scale: float = 0.0,
                 width: int = 32) -> dict:
    """Initial closure weights: hidden layers ~ N(0, hidden_scale^2); the output rows that update
    the hidden state ~ N(0, state_scale^2) and the bath-force row ~ N(0, force_scale^2) (both zero
    by default, which starts training from a quiet recurrence); output bias zero."""
    rs = Stream(seed, 5)
    shp = dict(CLOSURE_SHAPES)
    shp["W1"], shp["b1"], shp["W2"], shp["b2"], shp["W3"] = (width, 7), (width,), (width, width), (width,), (5, width)
    d = {}
    for k in ("W1", "b1", "W2", "b2"):
        d[k] = rs.normal(int(np.prod(shp[k]))).reshape(shp[k]) * hidden_scale
    w3 = rs.normal(5 * width).reshape(5, width)
    w3[:4] *= state_scale
    w3[4] *= force_scale
    d["W3"] = w3
    d["b3"] = np.zeros(5)
    return d


def closure_record(ntraj: int, nsteps: int, seed: int = 7, dt: float = 0.5):
    """Synthetic recorder output for trainer tests: E and P, [nsteps][ntraj] float32, P starting
    from rest.  Each trajectory is a smoothly switched-on, slowly decaying sinusoid with a random
    frequency in [0.8, 1.2], phase and time constants (stream 5); E is a second such signal."""
    rs = Stream(seed, 5)
    u = rs.uniform(6 * ntraj).reshape(6, ntraj)
    f = 0.8 + 0.4 * u[0]
    ph = 6.283185307179586 * u[1]
    tau = 20.0 + 40.0 * u[2]
    fe = 0.8 + 0.4 * u[3]
    phe = 6.283185307179586 * u[4]
    amp = 0.5 + u[5]
    t = (np.arange(nsteps) + 1.0)[:, None] * dt
    env = (1.0 - np.exp(-t / tau)) * np.exp(-t / (4.0 * tau))
    P = amp * np.sin(f * t + ph) * env
    P -= np.sin(ph) * amp * env * np.exp(-t)          # no jump at the start
    E = np.cos(fe * t + phe) * env
    return E.astype(np.float32), P.astype(np.float32)
