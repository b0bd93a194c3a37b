"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle on the same seeded inputs.

Bars: FP64 state <= 1e-12 relative L2, FP32 state <= 1e-5 (the FP32-state target
of the method's precision policy, measured as in tests/parity_util.py), DFT spectra
in FP64.  The long FP32 runs at each workload's own length are in
test_gpu_parity_long.py.
"""
import numpy as np
import pytest

from fdtdb_inputs import configs
from fdtdb_inputs.problem import (CLOSED, PERIODIC, PML, DftFlux, Drude, EnergyMonitor, LorentzBath, Problem,
                                  Source, box)
from tests.parity_util import TOL_F32, Lockstep

pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rel_fields(g, o, comps):
    """Per-component relative L2, with components far below the largest one measured against
    1e-6 of the largest norm (a field that is zero by symmetry has no relative error)."""
    ref = {c: o.field(c) for c in comps}
    big = max(np.linalg.norm(v) for v in ref.values())
    return {c: np.linalg.norm(g.field(c) - ref[c]) / max(np.linalg.norm(ref[c]), 1e-6 * big) for c in comps}


def run_pair(oracle_lib, p, steps=None, graph=0, dtype=None):
    from paper_2505_23963_amd import Grid
    n = p.steps if steps is None else steps
    print(f"[gpu] {p.name} n={p.n} steps={n} dtype={dtype or p.dtype} graph={graph}", flush=True)
    g = Grid(p, graph_chunk=graph, dtype=dtype)
    g.step(n)
    g.synchronize()
    o = oracle_lib.run(p, steps=n)
    return g, o


def fields_of(p):
    from fdtdb_inputs.problem import active_components
    e, h = active_components(p.ndim)
    return list(e) + list(h)


# ------------------------------------------------------------------------------------------ 1D
def test_config1_fp64_full(oracle_lib):
    """The 1D Fabry-Perot workload in full (2048 cells, N_b = 16, 20000 steps), FP64."""
    p = configs.config1_1d()
    g, o = run_pair(oracle_lib, p, graph=64)
    for c in fields_of(p):
        assert rel(g.field(c), o.field(c)) < 1e-12, c
    for mid in range(2):
        fg, fo = g.flux(mid), o.flux(mid)
        if mid == 0:
            assert rel(fg, fo) < 1e-11
        else:   # behind two opaque Drude mirrors: only compare at FP64 resolution of the inside flux
            assert np.max(np.abs(fg - fo)) < 1e-11 * np.max(np.abs(o.flux(0)))
    eg, eo = g.energy(0), o.energy(0)
    assert eg.shape == eo.shape
    assert np.max(np.abs(eg - eo)) < 1e-11 * np.abs(eo).max()
    for lvl in (0, 1):
        assert rel(g.polarization(1, 2, lvl), o.polarization(1, 2, lvl)) < 1e-12
        assert rel(g.bath(1, 2, lvl), o.bath(1, 2, lvl)) < 1e-11


@pytest.mark.parametrize("n", [1, 255, 257, 700])
def test_1d_ragged_sizes(oracle_lib, n):
    """Grids that are not a multiple of the block size, down to one cell."""
    p = Problem(name=f"rag{n}", ndim=1, n=(n, 1, 1), bc=(CLOSED, PERIODIC, PERIODIC), dtype="f64", steps=300)
    w, gm, k = configs.ohmic_bath(5, 0.8, 1.2, 1.0, seed=7)
    if n >= 10:
        p.materials.append(LorentzBath(box((n // 3, n - 2)), omega0=1.0, gamma0=0.01, eps_inf=1.2, sigma=0.05,
                                       n_bath=5, omega_j=w, gamma_j=gm, k_j=k))
        p.materials.append(Drude(box((1, 3)), omega_p=3.0, gamma=0.02, eps_inf=3.0))
    p.sources.append(Source(comp=2, box=box((0, 1)), omega_c=1.0, width=0.5))
    g, o = run_pair(oracle_lib, p)
    assert rel(g.field(2), o.field(2)) < 1e-12
    assert rel(g.field(4), o.field(4)) < 1e-12


# ------------------------------------------------------------------------------------------ 3D
def test_config2_crop_fp64(oracle_lib):
    """3D planar-cavity layout (z: PML | vac | Drude | LB N_b=8 random sigma | Drude | vac | PML), 10 x 12 crop."""
    p = configs.config2_3d(nx=10, ny=12, steps=220, nfreq=64, dtype="f64")
    g, o = run_pair(oracle_lib, p)
    errs = rel_fields(g, o, range(6))
    print("rel-L2 per component:", errs, flush=True)
    assert max(errs.values()) < 1e-12, errs
    assert rel(g.flux(0), o.flux(0)) < 1e-12
    assert rel(g.bath(1, 0, 0), o.bath(1, 0, 0)) < 1e-12


def test_config2_crop_fp32_graph(oracle_lib):
    """The same crop with FP32 state, replayed from captured graphs of 32 steps, checked every 110 steps
    (the FP32 measure of tests/parity_util.py)."""
    from paper_2505_23963_amd import Grid
    p = configs.config2_3d(nx=10, ny=12, steps=220, nfreq=64, dtype="f32")
    ls = Lockstep(Grid(p, graph_chunk=32), oracle_lib.Oracle(p), p).run(220, 110)
    ls.report()
    e, c = ls.worst()
    assert e < TOL_F32 and c < TOL_F32, (e, c)
    assert rel(ls.g.flux(0), ls.o.flux(0)) < TOL_F32


def test_3d_all_components_closed_box(oracle_lib):
    """A 3D box with closed and periodic axes, a transverse source and all six components driven."""
    rng = np.random.default_rng(3)
    n = (9, 7, 70)
    p = Problem(name="box3d", ndim=3, n=n, bc=(CLOSED, PERIODIC, CLOSED), dtype="f64", steps=150)
    w, gm, k = configs.ohmic_bath(7, 0.8, 1.2, 1.0, seed=11)
    lb = box((1, 8), (0, 7), (20, 50))
    p.materials += [LorentzBath(lb, omega0=1.0, gamma0=0.02, eps_inf=1.3, sigma_cells=rng.uniform(0.02, 0.1, 7 * 7 * 30),
                                n_bath=7, omega_j=w, gamma_j=gm, k_j=k),
                    Drude(box((0, 9), (0, 7), (55, 58)), omega_p=4.0, gamma=0.03, eps_inf=5.0)]
    p.sources += [Source(comp=1, box=box((2, 5), (1, 3), (10, 11)), omega_c=1.0, width=0.5),
                  Source(comp=2, box=box((4, 5), (3, 4), (12, 13)), omega_c=0.8, width=0.4, amplitude=0.7)]
    g, o = run_pair(oracle_lib, p)
    errs = rel_fields(g, o, range(6))
    assert max(errs.values()) < 1e-12, errs


@pytest.mark.parametrize("dtype,tol,nb", [("f64", 1e-12, 8), ("f32", 1e-5, 8), ("f64", 1e-12, 3)])
def test_3d_bath_layer_ragged_rows_and_chunks(oracle_lib, dtype, tol, nb):
    """A Lorentz-Bath block whose rows do not fill the 3D kernel's waves: an odd number of y rows (the
    last wave's upper half idle), a z extent of 75 (two full 32-cell chunks and a ragged one), and a
    block starting at z = 0 on a periodic z axis (the z - 1 neighbour wraps round); one and two groups
    of four bath modes."""
    rng = np.random.default_rng(5)
    n = (6, 9, 100)
    p = Problem(name="ragged3d", ndim=3, n=n, bc=(CLOSED, PERIODIC, PERIODIC), dtype=dtype, steps=200)
    w, gm, k = configs.ohmic_bath(nb, 0.8, 1.2, 1.0, seed=13)
    p.materials.append(LorentzBath(box((1, 5), (0, 9), (0, 75)), omega0=1.0, gamma0=0.01, eps_inf=1.2,
                                   sigma_cells=rng.uniform(0.02, 0.1, 4 * 9 * 75), n_bath=nb, omega_j=w,
                                   gamma_j=gm, k_j=k))
    p.sources += [Source(comp=0, box=box((2, 4), (1, 8), (80, 81)), omega_c=1.0, width=0.5),
                  Source(comp=2, box=box((3, 4), (4, 5), (90, 91)), omega_c=0.9, width=0.5, amplitude=0.5)]
    if dtype == "f32":
        from paper_2505_23963_amd import Grid
        ls = Lockstep(Grid(p), oracle_lib.Oracle(p), p).run(200, 100)
        ls.report()
        e, c = ls.worst()
        assert e < tol and c < tol, (e, c)
        return
    g, o = run_pair(oracle_lib, p)
    errs = rel_fields(g, o, range(6))
    assert max(errs.values()) < tol, errs
    assert rel(g.bath(0, 0, 0), o.bath(0, 0, 0)) < tol


# ------------------------------------------------------------------------------------------ 2D
# (the 2D TM workload with its N_b = 64 Lorentzian-form patch is compared over all 10 000 of its steps
# in tests/test_gpu_parity_long.py)


# ------------------------------------------------------------------------------------------ plain Lorentz
def _lorentz_problem(ndim, dtype, n_bath=0, steps=None):
    """A Lorentz slab (eq:Pz_1D_Lorentz; n_bath > 0 adds that many bath modes with zero coupling) between
    vacuum and CPML, driven by soft currents; in 3D every E component is driven and sigma varies per cell."""
    rng = np.random.default_rng(17)
    kw = {}
    if n_bath:
        kw = dict(n_bath=n_bath, omega_j=np.linspace(0.85, 1.15, n_bath), gamma_j=np.full(n_bath, 0.01),
                  k_j=np.zeros(n_bath))
    if ndim == 1:
        p = Problem(name=f"lorentz1d-nb{n_bath}", ndim=1, n=(600, 1, 1), bc=(PML, PERIODIC, PERIODIC),
                    pml_cells=(40, 0, 0), dtype=dtype, steps=steps or 3000)
        p.materials.append(LorentzBath(box((250, 400)), omega0=1.0, gamma0=0.02, eps_inf=1.5, sigma=0.05, **kw))
        p.sources.append(Source(comp=2, box=box((100, 101)), omega_c=1.0, width=0.4))
        p.dfts.append(DftFlux(0, box((500, 501)), np.linspace(0.6, 1.4, 41)))
    else:
        p = Problem(name=f"lorentz3d-nb{n_bath}", ndim=3, n=(8, 6, 160), bc=(PERIODIC, PERIODIC, PML),
                    pml_cells=(0, 0, 16), dtype=dtype, steps=steps or 800)
        p.materials.append(LorentzBath(box((0, 8), (0, 6), (60, 110)), omega0=1.0, gamma0=0.02, eps_inf=1.5,
                                       sigma_cells=rng.uniform(0.02, 0.1, 8 * 6 * 50), **kw))
        p.sources += [Source(comp=0, box=box((0, 8), (0, 6), (30, 31)), omega_c=1.0, width=0.4),
                      Source(comp=1, box=box((2, 5), (1, 4), (35, 36)), omega_c=0.9, width=0.5, amplitude=0.5),
                      Source(comp=2, box=box((4, 5), (3, 4), (40, 41)), omega_c=1.1, width=0.5, amplitude=0.3)]
        p.dfts.append(DftFlux(2, box((0, 8), (0, 6), (130, 131)), np.linspace(0.6, 1.4, 17)))
    return p


@pytest.mark.parametrize("ndim", [1, 3])
def test_plain_lorentz_fp64(oracle_lib, ndim):
    """Plain Lorentz media (no bath, eq:Pz_1D_Lorentz) against the oracle in FP64: fields, both
    polarization levels and the flux spectrum."""
    p = _lorentz_problem(ndim, "f64")
    g, o = run_pair(oracle_lib, p)
    errs = rel_fields(g, o, fields_of(p))
    print("rel-L2 per component:", errs, flush=True)
    assert max(errs.values()) < 1e-12, errs
    e = (2,) if ndim == 1 else (0, 1, 2)
    for c in e:
        for lvl in (0, 1):
            assert rel(g.polarization(0, c, lvl), o.polarization(0, c, lvl)) < 1e-12, (c, lvl)
    assert rel(g.flux(0), o.flux(0)) < 1e-12


@pytest.mark.parametrize("ndim", [1, 3])
def test_plain_lorentz_fp32(oracle_lib, ndim):
    """The same media with FP32 state (the FP32 measure of tests/parity_util.py, five checkpoints)."""
    from paper_2505_23963_amd import Grid
    p = _lorentz_problem(ndim, "f32")
    ls = Lockstep(Grid(p), oracle_lib.Oracle(p), p).run(p.steps, p.steps // 5)
    ls.report()
    e, c = ls.worst()
    assert e < TOL_F32 and c < TOL_F32, (e, c)
    assert rel(ls.g.flux(0), ls.o.flux(0)) < TOL_F32


@pytest.mark.parametrize("ndim,n_bath,dtype", [(1, 4, "f64"), (1, 4, "f32"), (3, 4, "f32"), (3, 16, "f32"),
                                               (3, 8, "f64")])
def test_zero_coupling_equals_lorentz_on_gpu(ndim, n_bath, dtype):
    """k_j = 0 makes eq:Pz_update-LB the Lorentz update eq:Pz_1D_Lorentz (c_j = 0, A = 1 + g0 dt/2, no bath
    force): a Lorentz-Bath medium with zero couplings, run by the bath kernels (load-first, and the
    component-split kernel for N_b = 16 in 3D), advances like the plain Lorentz medium to within one
    unit in the last place of the state's precision, and its bath coordinates stay zero."""
    from paper_2505_23963_amd import Grid
    a = Grid(_lorentz_problem(ndim, dtype))
    b = Grid(_lorentz_problem(ndim, dtype, n_bath=n_bath))
    steps = a.p.steps
    a.step(steps)
    b.step(steps)
    ft = np.float32 if dtype == "f32" else np.float64
    worst = 0.0
    e = (2,) if ndim == 1 else (0, 1, 2)
    for c in fields_of(a.p):
        x, y = a.field(c), b.field(c)
        ulp = np.spacing(np.abs(x).astype(ft)).astype(np.float64)
        worst = max(worst, float(np.max(np.abs(x - y) / ulp)))
    for c in e:
        x, y = a.polarization(0, c, 0), b.polarization(0, c, 0)
        worst = max(worst, float(np.max(np.abs(x - y) / np.spacing(np.abs(x).astype(ft)).astype(np.float64))))
        assert not np.any(b.bath(0, c, 0)), c
    print(f"[gpu] zero coupling vs Lorentz: largest difference {worst:.1f} ulp", flush=True)
    assert worst <= 1.0


# ------------------------------------------------------------------------------------------ properties
def test_energy_conservation_on_gpu(oracle_lib):
    """Lossless closed box on the GPU (FP64): the exact discrete energy stays constant."""
    p = Problem(name="econs", ndim=2, n=(40, 30, 1), bc=(CLOSED, PERIODIC, PERIODIC), dtype="f64", steps=3000)
    w = np.array([0.8, 0.95, 1.05, 1.2])
    p.materials.append(LorentzBath(box((5, 35), (0, 30)), omega0=1.0, gamma0=0.0, eps_inf=1.5, sigma=0.08,
                                   n_bath=4, omega_j=w, gamma_j=np.zeros(4), k_j=np.array([0.05, 0.1, 0.08, 0.04])))
    p.sources.append(Source(comp=2, box=box((20, 21), (10, 20)), omega_c=1.0, width=2.0))
    p.energies.append(EnergyMonitor(box((0, 40), (0, 30)), every=5))
    g, o = run_pair(oracle_lib, p)
    e = g.energy(0).sum(axis=1)
    assert np.max(np.abs(e[4:] - e[4])) / e[4] < 1e-11
    assert np.max(np.abs(g.energy(0) - o.energy(0))) < 1e-11 * e[4]


def test_graph_replay_matches_direct():
    """Graph replays (with eager work and syncs between them) equal direct launches bitwise."""
    from paper_2505_23963_amd import Grid
    p = configs.config2_3d(nx=6, ny=5, steps=0, nfreq=16)
    print("[gpu] graph vs direct", flush=True)
    a = Grid(p)
    b = Grid(p, graph_chunk=32)
    for rep in range(3):
        a.step(64)
        b.step(64)
        a.synchronize()
        b.synchronize()
        for c in range(6):
            assert np.array_equal(a.field(c), b.field(c)), (rep, c)
    assert np.array_equal(a.flux(0), b.flux(0))


def test_rerun_bitwise_identical():
    from paper_2505_23963_amd import Grid
    p = configs.config2_3d(nx=6, ny=5, steps=100, nfreq=16)
    out = []
    for _ in range(2):
        g = Grid(p)
        g.step(p.steps)
        out.append((g.field(0), g.flux(0)))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


# ------------------------------------------------------------------------------------------ boundary errors
def test_validator_and_errors():
    from paper_2505_23963_amd import FdtdbError, Grid
    from paper_2505_23963_amd.fdtdb import E_INVALID, E_STATE, E_UNSTABLE, E_DIVERGED
    base = dict(name="err", ndim=1, n=(100, 1, 1), bc=(PML, PERIODIC, PERIODIC), pml_cells=(10, 0, 0), dtype="f64")
    # Drude mirror with eps_inf = 1 at omega_p = 10 is unstable at Courant 0.5
    p = Problem(**base)
    p.materials.append(Drude(box((40, 50)), omega_p=10.0, gamma=0.01, eps_inf=1.0))
    with pytest.raises(FdtdbError) as ei:
        Grid(p)
    assert ei.value.status == E_UNSTABLE
    # dispersive material inside the CPML
    p = Problem(**base)
    p.materials.append(LorentzBath(box((5, 20)), omega0=1.0, gamma0=0.0, eps_inf=1.0, sigma=0.05))
    with pytest.raises(FdtdbError) as ei:
        Grid(p)
    assert ei.value.status == E_INVALID
    # overlapping boxes
    p = Problem(**base)
    p.materials += [Drude(box((40, 50)), omega_p=1.0, gamma=0.01, eps_inf=2.0),
                    Drude(box((45, 55)), omega_p=1.0, gamma=0.01, eps_inf=2.0)]
    with pytest.raises(FdtdbError) as ei:
        Grid(p)
    assert ei.value.status == E_INVALID
    # Courant above the 3D limit
    with pytest.raises(FdtdbError) as ei:
        Grid(Problem(name="c", ndim=3, n=(4, 4, 4), courant=0.6))
    assert ei.value.status == E_UNSTABLE
    # materials after the first step
    from paper_2505_23963_amd.fdtdb import Box, lib
    import ctypes as C
    g = Grid(Problem(**base))
    g.step(1)
    b = Box()
    b.lo[:] = [30, 0, 0]
    b.hi[:] = [40, 1, 1]
    assert lib().fdtdb_set_eps_inf(g.h, C.byref(b), 2.0, None) == E_STATE
    # watchdog: a NaN planted from the host is reported by synchronize
    bad = np.zeros(100)
    bad[50] = np.nan
    g.set_field(2, bad)
    g.step(2)
    with pytest.raises(FdtdbError) as ei:
        g.synchronize()
    assert ei.value.status == E_DIVERGED


@pytest.mark.parametrize("eps_factor,ok", [(1.03, True), (0.97, False)])
def test_validator_drude_bound_matches_propagator(oracle_lib, eps_factor, ok):
    """The library's Drude acceptance agrees with the oracle's brute-force propagator spectrum."""
    from paper_2505_23963_amd import FdtdbError, Grid
    from tests.test_oracle_pins import one_step_map, _periodic_1d
    wp = 6.0
    eps = 0.25 * (wp ** 2 + 4.0) / 4.0 * eps_factor
    lam = np.abs(np.linalg.eigvals(one_step_map(oracle_lib, _periodic_1d(8, [Drude(box((0, 8)), omega_p=wp,
                                                                                    gamma=0.0, eps_inf=eps)]))))
    stable = lam.max() < 1 + 1e-6
    assert stable == ok
    p = Problem(name="v", ndim=1, n=(8, 1, 1), bc=(PERIODIC, PERIODIC, PERIODIC), dtype="f64")
    p.materials.append(Drude(box((0, 8)), omega_p=wp, gamma=0.0, eps_inf=eps))
    if ok:
        Grid(p)
    else:
        with pytest.raises(FdtdbError):
            Grid(p)


# (the full 256 x 256 x 512 workload for 200 steps is in tests/test_gpu_parity_long.py)


# ------------------------------------------------------------------------------------------ CPML
def _cpml_cases():
    """A pulse launched next to the upper absorbing layer, run until it has crossed both layers:
    every E-type and H-type node with nonzero grading carries psi.  Layer thicknesses both
    divisible and not divisible by 4 (the vector kernels run along z in 3D and y in 2D)."""
    out = []
    for L in (8, 10):
        p = Problem(name=f"cpml1d-L{L}", ndim=1, n=(160, 1, 1), bc=(PML, PERIODIC, PERIODIC), pml_cells=(L, 0, 0),
                    dtype="f64", steps=400)
        p.materials.append(Drude(box((60, 70)), omega_p=0.0, gamma=0.0, eps_inf=4.0))
        p.sources.append(Source(comp=2, box=box((140, 141)), omega_c=1.0, width=0.6))
        out.append(p)
        p = Problem(name=f"cpml2d-L{L}", ndim=2, n=(40, 64, 1), bc=(PML, PML, PERIODIC), pml_cells=(L, L, 0),
                    dtype="f64", steps=160)
        p.sources.append(Source(comp=2, box=box((28, 29), (48, 49)), omega_c=1.0, width=0.6))
        out.append(p)
        p = Problem(name=f"cpml3d-L{L}", ndim=3, n=(6, 8, 64), bc=(PERIODIC, PERIODIC, PML), pml_cells=(0, 0, L),
                    dtype="f64", steps=200)
        p.sources.append(Source(comp=0, box=box((0, 6), (0, 8), (50, 51)), omega_c=1.0, width=0.6))
        out.append(p)
        # absorbing layers on all three axes: edge, corner and interior regions, each with its own set
        # of psi terms (per cell across x and y, the per-row tail of the z layer where it applies)
        p = Problem(name=f"cpml3d-all-L{L}", ndim=3, n=(28, 24, 40), bc=(PML, PML, PML), pml_cells=(L, L, L),
                    dtype="f64", steps=160)
        p.sources.append(Source(comp=1, box=box((18, 19), (14, 15), (26, 27)), omega_c=1.0, width=0.6))
        p.sources.append(Source(comp=2, box=box((12, 13), (11, 12), (30, 31)), omega_c=0.8, width=0.5, amplitude=0.5))
        out.append(p)
    return out


@pytest.mark.parametrize("p", _cpml_cases(), ids=lambda p: p.name)
def test_cpml_layers_fp64(oracle_lib, p):
    g, o = run_pair(oracle_lib, p)
    if "all" in p.name:
        # point sources: the H components are 30-200x smaller than E and formed from differences of E,
        # so each component is measured against the largest component's norm (FP64 rounding of E is
        # 1e-12 of H's own norm near the sources)
        ref = {c: o.field(c) for c in fields_of(p)}
        big = max(np.linalg.norm(v) for v in ref.values())
        errs = {c: np.linalg.norm(g.field(c) - v) / big for c, v in ref.items()}
    else:
        errs = rel_fields(g, o, fields_of(p))
    print("rel-L2 per component:", errs, flush=True)
    assert max(errs.values()) < 1e-12, errs


# ------------------------------------------------------------------- 3D baths of more than 8 modes
@pytest.mark.parametrize("case", ["config5", "config2_nb12"])
def test_3d_large_baths_component_split_fp64(oracle_lib, case):
    """3D baths whose components x mode groups exceed 6 take the one-(component, cell)-per-thread kernel:
    the 512^3 layout (N_b = 16, Gaussian-profile plane source) on an 8 x 8 crop, and the planar cavity
    with N_b = 12, against the oracle in FP64.  The Gaussian-profile source drives E_y, E_z, H_x and H_z
    only through diffraction (1e-8 to 1e-3 of the dominant norm): components below 1 % of the largest
    are measured against 1 % of it."""
    if case == "config5":
        p = configs.config5_3d_large(nx=8, ny=8, steps=500, nfreq=32, dtype="f64")
    else:
        p = configs.config2_3d(nx=10, ny=12, steps=220, nfreq=64, nb=12, dtype="f64")
    g, o = run_pair(oracle_lib, p)
    ref = {c: o.field(c) for c in range(6)}
    big = max(np.linalg.norm(v) for v in ref.values())
    errs = {c: np.linalg.norm(g.field(c) - ref[c]) / max(np.linalg.norm(ref[c]), 1e-2 * big) for c in range(6)}
    print("rel-L2 per component:", errs, flush=True)
    assert max(errs.values()) < 1e-12, errs
    assert rel(g.flux(0), o.flux(0)) < 1e-12
    mi = 0 if case == "config5" else 1
    for get in (lambda x, c: x.polarization(mi, c, 0), lambda x, c: x.bath(mi, c, 1)):
        r = [get(o, c) for c in range(3)]
        top = max(np.linalg.norm(v) for v in r)
        for c in range(3):
            assert np.linalg.norm(get(g, c) - r[c]) / max(np.linalg.norm(r[c]), 1e-2 * top) < 1e-12, c


def test_3d_component_split_nb12_fp32(oracle_lib):
    """The planar cavity with N_b = 12 (component-split kernel, three mode groups) in FP32."""
    from paper_2505_23963_amd import Grid
    p = configs.config2_3d(nx=10, ny=12, steps=440, nfreq=64, nb=12, dtype="f32")
    ls = Lockstep(Grid(p), oracle_lib.Oracle(p), p).run(440, 110)
    ls.report()
    e, c = ls.worst()
    assert e < TOL_F32 and c < TOL_F32, (e, c)
    assert rel(ls.g.flux(0), ls.o.flux(0)) < TOL_F32


def test_two_row_waves_bitwise_equal_one_row_kernel():
    """The 3D Lorentz-Bath kernel's two-row wave layout (taken without energy sampling) and its
    one-row layout (taken when an energy monitor samples the layer) advance the N_b = 8 layer
    identically, bit for bit, on a crop with an odd number of rows."""
    from paper_2505_23963_amd import Grid
    p = configs.config2_3d(nx=6, ny=7, steps=300, nfreq=8, dtype="f32")
    q = configs.config2_3d(nx=6, ny=7, steps=300, nfreq=8, dtype="f32")
    q.energies.append(EnergyMonitor(box((0, 6), (0, 7), (56, 456)), every=1))
    a, b = Grid(p), Grid(q)
    a.step(300)
    b.step(300)
    for c in range(6):
        assert np.array_equal(a.field(c), b.field(c)), c
    for c in range(3):
        assert np.array_equal(a.polarization(1, c, 0), b.polarization(1, c, 0)), c
        assert np.array_equal(a.bath(1, c, 0), b.bath(1, c, 0)), c


def test_component_split_bitwise_equals_per_cell_kernel():
    """The component-split kernel and the per-cell kernel (taken when an energy monitor samples the
    region) advance the N_b = 16 layer identically, bit for bit."""
    from paper_2505_23963_amd import Grid
    p = configs.config5_3d_large(nx=8, ny=8, steps=300, nfreq=8, dtype="f32")
    q = configs.config5_3d_large(nx=8, ny=8, steps=300, nfreq=8, dtype="f32")
    q.energies.append(EnergyMonitor(box((0, 8), (0, 8), (140, 370)), every=1))
    a, b = Grid(p), Grid(q)
    a.step(300)
    b.step(300)
    for c in range(6):
        assert np.array_equal(a.field(c), b.field(c)), c
    for c in range(3):
        assert np.array_equal(a.bath(0, c, 0), b.bath(0, c, 0)), c


# ------------------------------------------------------------------------------------------ read-out, watchdog
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_field_readout_to_device_equals_host(dtype):
    """fdtdb_get_field with a device destination writes the same FP64 values as the host read-out."""
    import torch
    from paper_2505_23963_amd import Grid
    p = configs.config2_3d(nx=6, ny=5, steps=80, nfreq=8, dtype=dtype)
    g = Grid(p)
    g.step(80)
    for c in range(6):
        t = torch.full((p.cells,), float("nan"), dtype=torch.float64, device="cuda")
        g.field_into(c, t.data_ptr())
        assert np.array_equal(t.cpu().numpy().reshape(p.n), g.field(c)), c


def _watchdog_box(every=5):
    p = Problem(name="wd", ndim=1, n=(200, 1, 1), bc=(CLOSED, PERIODIC, PERIODIC), dtype="f32", steps=0)
    p.materials.append(LorentzBath(box((80, 140)), omega0=1.0, gamma0=0.0, eps_inf=1.0, sigma=0.05, n_bath=4,
                                   omega_j=np.linspace(0.9, 1.1, 4), gamma_j=np.zeros(4), k_j=np.full(4, 0.05)))
    p.sources.append(Source(comp=2, box=box((40, 41)), omega_c=1.0, width=0.5))
    p.energies.append(EnergyMonitor(box((0, 200)), every=every))
    return p


def test_watchdog_energy_growth():
    """A lossless closed box with a whole-grid energy monitor runs clean; energy planted from the host after
    the source has ended (a field ten times larger) is reported as growth by synchronize (E_DIVERGED)."""
    from paper_2505_23963_amd import FdtdbError, Grid
    from paper_2505_23963_amd.fdtdb import E_DIVERGED
    g = Grid(_watchdog_box())
    g.step(2000)
    g.synchronize()                      # the source ended at step 40; energy exactly conserved since
    g.set_field(2, 10.0 * g.field(2))
    g.step(10)
    with pytest.raises(FdtdbError) as ei:
        g.synchronize()
    assert ei.value.status == E_DIVERGED and "energy" in str(ei.value)


def test_watchdog_quiet_on_absorbing_and_lossy_grids():
    """A monitor over every cell inside the CPML layers, on a grid whose energy leaves through those
    layers and decays in the bath, never trips the watchdog (2D grid with CPML on every side and a
    Lorentzian-form N_b = 64 patch, FP32)."""
    from paper_2505_23963_amd import Grid
    p = configs.config4_2d(n=160, patch=(60, 110), steps=0, nfreq=8, src_x=40, flux_x=125)
    p.energies.append(EnergyMonitor(box((32, 128), (32, 128)), every=10))
    g = Grid(p)
    for _ in range(6):
        g.step(500)
        g.synchronize()
    e = g.energy(0).sum(axis=1)
    assert e[-1] < 0.2 * e.max()
