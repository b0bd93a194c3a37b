"""Bloch-periodic grids on the GPU (fdtdb_pair_bloch): the real and imaginary parts of complex fields as
two device grids coupled at the Bloch wrap, against the oracle's Bloch pairs (tests/test_bloch_oracle.py
pins those) and against the lattice transfer matrix at oblique incidence."""
import numpy as np
import pytest

from fdtdb_inputs.problem import (PERIODIC, PML, DftFlux, Drude, EnergyMonitor, LorentzBath, MultiPole, Problem,
                                  Source, box)
from tests.parity_util import TOL_F32

pytestmark = pytest.mark.gpu
DT = 0.5


def _problem_2d(dtype="f64", phase=0.9, steps=600, n_bath=8, energy=True):
    """2D TM, CPML along x, Bloch along y (16 cells): a Lorentz-Bath slab (8 modes), a Drude film, a
    Lorentz + Drude multi-term block over part of the period, a source with a complex profile."""
    nx, ny = 140, 16
    rs = np.random.default_rng(21)
    p = Problem(name="bloch-2d", ndim=2, n=(nx, ny, 1), bc=(PML, PERIODIC, PERIODIC), pml_cells=(20, 0, 0),
                dtype=dtype, steps=steps, bloch=(0.0, phase, 0.0))
    p.materials += [
        LorentzBath(box((50, 80), (0, ny)), omega0=1.0, gamma0=0.01, eps_inf=1.3, sigma=0.08, n_bath=n_bath,
                    omega_j=np.linspace(0.85, 1.15, n_bath), gamma_j=np.full(n_bath, 0.02),
                    k_j=np.full(n_bath, 0.48 / n_bath)),
        Drude(box((100, 103), (0, ny)), omega_p=3.0, gamma=0.02, eps_inf=2.0),
        MultiPole(box((85, 95), (3, 11)), eps_inf=1.5, kinds=("lorentz", "drude"), omega=(1.2, 0.6),
                  gamma=(0.03, 0.02), sigma=(0.2, 0.0)),
    ]
    ky = phase / ny
    j = np.arange(ny)
    p.sources.append(Source(comp=2, box=box((30, 31), (0, ny)), omega_c=1.0, width=0.4,
                            profile=np.cos(ky * j) * rs.uniform(0.8, 1.2, ny),
                            profile_im=np.sin(ky * j) * rs.uniform(0.8, 1.2, ny)))
    p.dfts.append(DftFlux(0, box((115, 116), (0, ny)), np.linspace(0.6, 1.4, 9)))
    if energy:
        p.energies.append(EnergyMonitor(box((20, 120), (0, ny)), every=25))
    return p


def _problem_3d(dtype="f64", steps=300):
    """3D, Bloch along x and y (phases 0.5 and -1.3), CPML along z: a Lorentz-Bath slab of 16 modes (the
    component-split kernel on a real grid) and a Drude film."""
    nx, ny, nz = 6, 8, 72
    p = Problem(name="bloch-3d", ndim=3, n=(nx, ny, nz), bc=(PERIODIC, PERIODIC, PML), pml_cells=(0, 0, 12),
                dtype=dtype, steps=steps, bloch=(0.5, -1.3, 0.0))
    w, g, k = np.linspace(0.8, 1.2, 16), np.full(16, 0.02), np.full(16, 0.05)
    p.materials += [
        LorentzBath(box((0, nx), (0, ny), (30, 50)), omega0=1.0, gamma0=0.0, eps_inf=1.0, sigma=0.05, n_bath=16,
                    omega_j=w, gamma_j=g, k_j=k),
        Drude(box((0, nx), (0, ny), (55, 57)), omega_p=4.0, gamma=0.01, eps_inf=10.0),
    ]
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    ph = 0.5 / nx * X - 1.3 / ny * Y
    for comp in (0, 1):
        p.sources.append(Source(comp=comp, box=box((0, nx), (0, ny), (20, 21)), omega_c=1.0, width=0.4,
                                profile=np.cos(ph).reshape(nx, ny, 1) * (1 + comp),
                                profile_im=np.sin(ph).reshape(nx, ny, 1) * (1 + comp)))
    p.dfts.append(DftFlux(2, box((0, nx), (0, ny), (62, 63)), np.linspace(0.6, 1.4, 9)))
    p.energies.append(EnergyMonitor(box((0, nx), (0, ny), (12, 60)), every=20))
    return p


def _compare(g, o, p, tol, steps):
    g.step(steps)
    g.synchronize()
    o.step(steps)
    worst = {}
    from fdtdb_inputs.problem import active_components
    ec, hc = active_components(p.ndim)
    for c in (*ec, *hc):
        ref = o.field(c)
        worst[f"F{c}"] = np.linalg.norm(g.field(c) - ref) / np.linalg.norm(ref)
    for mi, m in enumerate(p.materials):
        kind = type(m).__name__
        for c in ec:
            if kind == "MultiPole":
                # Lorentz terms: level 0 as stored; Drude terms by increment (polarization(level 0) - level 1 on the
                # oracle, the stored increment on the GPU)
                for t, kd in enumerate(m.kinds):
                    ref = o.pole(mi, c, t, 0) - (o.pole(mi, c, t, 1) if kd == "drude" else 0)
                    worst[f"M{mi}.{c}.{t}"] = np.linalg.norm(g.pole(mi, c, t, 0) - ref) / np.linalg.norm(ref)
                continue
            if kind == "Drude":
                continue
            ref = o.polarization(mi, c, 0)
            worst[f"P{mi}.{c}"] = np.linalg.norm(g.polarization(mi, c, 0) - ref) / np.linalg.norm(ref)
            if getattr(m, "n_bath", 0):
                ref = o.bath(mi, c, 0)
                worst[f"Y{mi}.{c}"] = np.linalg.norm(g.bath(mi, c, 0) - ref) / np.linalg.norm(ref)
    fo = o.flux(0)
    worst["flux"] = np.max(np.abs(g.flux(0) - fo)) / np.max(np.abs(fo))
    if p.energies:
        eo = o.energy(0)
        worst["energy"] = np.max(np.abs(g.energy(0) - eo)) / np.max(np.abs(eo))
    for k, v in worst.items():
        print(f"  {k}: {v:.2e}", flush=True)
    bad = {k: v for k, v in worst.items() if not v < tol}
    assert not bad, bad


def test_bloch_2d_fp64_equals_oracle(oracle_lib):
    from paper_2505_23963_amd import Grid
    p = _problem_2d()
    print(f"[gpu] bloch 2d fp64 {p.n}, phase {p.bloch}", flush=True)
    _compare(Grid(p), oracle_lib.Oracle(p), p, 1e-12, 600)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", TOL_F32)])
def test_bloch_2d_wide_bath_without_energy(oracle_lib, dtype, tol):
    """64 bath modes and no energy monitor: the slab's wrap rows take the load-first bath kernel in its
    coefficient-table form (16 mode groups), the one the full-size 2D Bloch grid runs."""
    from paper_2505_23963_amd import Grid
    p = _problem_2d(dtype=dtype, n_bath=64, energy=False)
    print(f"[gpu] bloch 2d {dtype} {p.n}, 64 modes, no energy monitor", flush=True)
    _compare(Grid(p), oracle_lib.Oracle(p), p, tol, 600)


def test_bloch_3d_fp64_equals_oracle(oracle_lib):
    from paper_2505_23963_amd import Grid
    p = _problem_3d()
    print(f"[gpu] bloch 3d fp64 {p.n}, phases {p.bloch}", flush=True)
    _compare(Grid(p), oracle_lib.Oracle(p), p, 1e-12, 300)


def test_bloch_2d_fp32_state(oracle_lib):
    from paper_2505_23963_amd import Grid
    p = _problem_2d(dtype="f32")
    print(f"[gpu] bloch 2d fp32 {p.n}", flush=True)
    _compare(Grid(p), oracle_lib.Oracle(p), p, TOL_F32, 600)


def test_bloch_zero_phase_equals_periodic_grid():
    """phi = 0 (the pair takes the generic kernels) equals the plain periodic grid (vector kernels) to FP64
    rounding; the imaginary part without a source stays zero."""
    from paper_2505_23963_amd import Grid
    p = _problem_2d(phase=0.0, steps=400)
    p.sources[0].profile_im = None
    g = Grid(p)
    q = _problem_2d(phase=0.0, steps=400)
    q.sources[0].profile_im = None
    q.bloch = None
    r = Grid(q)
    g.step(400)
    r.step(400)
    for c in (2, 3, 4):
        a, b = g.field(c), r.field(c)
        assert not np.any(a.imag)
        assert np.linalg.norm(a.real - b) < 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("which", ["lorentz_bath", "drude"])
def test_bloch_oblique_slab_transmission_lattice_tmm(which):
    """The oblique-incidence transmission of the oracle pin, on the GPU (FP64), against the lattice transfer
    matrix with the transverse term."""
    from oracle.closed_form import chi_discrete, lattice_transmission
    from paper_2505_23963_amd import Grid
    ky, ny, nx = 0.4, 2, 800
    if which == "lorentz_bath":
        w = np.linspace(0.75, 1.25, 26)
        wj, gj, kj = np.linspace(0.85, 1.15, 8), np.full(8, 0.02), np.full(8, 0.06)
        mats = [LorentzBath(box((300, 400), (0, ny)), omega0=1.0, gamma0=0.02, eps_inf=1.2, sigma=0.05, n_bath=8,
                            omega_j=wj, gamma_j=gj, k_j=kj)]
        chi = chi_discrete(w, DT, 1.0, 0.02, 0.05, wj, gj, kj)
        eps, L, steps = 1.2, 100, 30000
    else:
        w = np.linspace(0.75, 1.25, 21)
        mats = [Drude(box((300, 302), (0, ny)), omega_p=4.0, gamma=0.01, eps_inf=10.0)]
        chi = chi_discrete(w, DT, 4.0, 0.01, 1.0, drude=True)
        eps, L, steps = 10.0, 2, 16000

    def run(ms):
        p = Problem(name="bloch-tmm", ndim=2, n=(nx, ny, 1), bc=(PML, PERIODIC, PERIODIC), pml_cells=(40, 0, 0),
                    dtype="f64", steps=steps, bloch=(0.0, ny * ky, 0.0))
        p.materials += ms
        j = np.arange(ny)
        p.sources.append(Source(comp=2, box=box((100, 101), (0, ny)), omega_c=1.0, width=0.12,
                                profile=np.cos(ky * j), profile_im=np.sin(ky * j)))
        p.dfts.append(DftFlux(0, box((nx - 150, nx - 149), (0, ny)), w))
        g = Grid(p)
        g.step(steps)
        return g.flux(0)
    T = run(mats) / run([])
    ref = lattice_transmission(w, DT, np.full(L, eps), np.tile(chi, (L, 1)), ky=ky)
    err = np.max(np.abs(T - ref))
    print(f"  {which}: max |T_gpu - T_tmm| = {err:.2e}", flush=True)
    assert err < 1e-6


def test_bloch_pair_validation():
    import ctypes as C

    from paper_2505_23963_amd import Grid
    from paper_2505_23963_amd.fdtdb import E_INVALID, E_STATE, FdtdbError, lib
    p = _problem_2d(steps=10)
    g = Grid(p)
    # the imaginary part steps only through the real part
    assert lib().fdtdb_step(g.h_im, 1) == E_STATE
    assert lib().fdtdb_dft_flux(g.h_im, 0, np.zeros(9).ctypes.data_as(C.POINTER(C.c_double)), None) == E_STATE
    g.step(10)
    # a phase needs a periodic axis; a flux plane normal to a Bloch axis may not sit at its first cell
    q = _problem_2d(steps=10)
    q.bloch = (0.3, 0.9, 0.0)
    with pytest.raises(FdtdbError) as e:
        Grid(q)
    assert e.value.status == E_INVALID
    q = _problem_2d(steps=10)
    q.bc = (PERIODIC, PERIODIC, PERIODIC)
    q.pml_cells = (0, 0, 0)
    q.bloch = (0.4, 0.9, 0.0)
    q.dfts[0] = DftFlux(0, box((0, 1), (0, 16)), np.linspace(0.6, 1.4, 9))
    with pytest.raises(FdtdbError) as e:
        Grid(q)
    assert e.value.status == E_INVALID
    # no learned closures on Bloch grids
    with pytest.raises(ValueError):
        Grid(_problem_2d(steps=10), closures={0: {"weights": np.zeros(1477), "scales": (1, 1, 1, 1)}})
    h = Grid(_problem_2d(steps=10))
    w = np.zeros(1477, np.float32)
    sc = np.ones(4)
    assert lib().fdtdb_set_bath_closure(h.h, h.mat_ids[0], w.ctypes.data_as(C.POINTER(C.c_float)), 32,
                                        sc.ctypes.data_as(C.POINTER(C.c_double))) == E_STATE
    # once one part is destroyed the other cannot step
    r = Grid(_problem_2d(steps=10))
    lib().fdtdb_destroy_grid(r.h_im)
    r.h_im = None
    assert lib().fdtdb_step(r.h, 1) == E_STATE
