"""Pins of the oracle's Bloch-periodic grids (complex fields as two coupled real parts).

The paper's 2D runs are Bloch-periodic along y (Appendix, "Simulation details"); a grid with phase
phi_a on axis a carries complex fields with f(r + n_a e_a) = exp(i phi_a) f(r).  Pinned here against
what the definition and the lattice fix, not against the oracle itself:
  * phase 0 is the plain periodic grid (real part bitwise equal, imaginary part zero);
  * a lattice Bloch plane wave exp(i (kx x + ky y)) with ky n_y = phi (mod 2 pi) keeps its shape and
    its amplitude follows the exact two-step recurrence c' = (2 - dt^2 K^2) c - c_prev of the Yee
    scheme, K^2 = 4 sin^2(kx/2) + 4 sin^2(ky/2) -- a wrong sign or a missing phase at either wrap
    (the E update reads H below the lower end, the H update reads E past the upper end) breaks it;
  * oblique-incidence transmission through Lorentz-Bath and Drude slabs equals the lattice transfer
    matrix with the transverse term -4 sin^2(ky/2) (closed_form.lattice_transmission with ky).
"""
import numpy as np
import pytest

from fdtdb_inputs.problem import PERIODIC, PML, DftFlux, Drude, LorentzBath, Problem, Source, box

DT = 0.5


def _slab_problem(nx, ny, mats, w, phase, steps, ky=None, with_src=True, width=0.2):
    p = Problem(name="bloch", ndim=2, n=(nx, ny, 1), bc=(PML, PERIODIC, PERIODIC), pml_cells=(40, 0, 0),
                dtype="f64", steps=steps, bloch=None if phase is None else (0.0, phase, 0.0))
    p.materials += mats
    if with_src:
        j = np.arange(ny)
        kyy = (phase or 0.0) / ny if ky is None else ky
        p.sources.append(Source(comp=2, box=box((100, 101), (0, ny)), omega_c=1.0, width=width,
                                profile=np.cos(kyy * j), profile_im=np.sin(kyy * j)))
    p.dfts.append(DftFlux(0, box((nx - 150, nx - 149), (0, ny)), w))
    return p


def test_bloch_zero_phase_is_the_periodic_grid(oracle_lib):
    """phi = 0: the real part is the plain periodic grid, bit for bit, and the imaginary part, with no
    source of its own, stays exactly zero."""
    w = np.linspace(0.7, 1.3, 7)
    rs = np.random.default_rng(3)   # any real profile along y
    slab = LorentzBath(box((120, 160), (0, 6)), omega0=1.0, gamma0=0.01, eps_inf=1.5, sigma=0.05, n_bath=4,
                       omega_j=np.linspace(0.9, 1.1, 4), gamma_j=np.full(4, 0.01), k_j=np.full(4, 0.05))
    prof = rs.uniform(0.5, 1.5, 6)
    runs = []
    for phase in (None, 0.0):
        p = _slab_problem(300, 6, [slab], w, phase, 400)
        p.sources[0].profile, p.sources[0].profile_im = prof, None
        o = oracle_lib.Oracle(p)
        o.step(400)
        runs.append(o)
    plain, bl = runs
    for comp in (2, 3, 4):
        assert np.array_equal(plain.field(comp), bl.field(comp).real)
        assert not np.any(bl.field(comp).imag)
    assert np.array_equal(plain.bath(0, 2), bl.bath(0, 2).real)
    assert np.array_equal(plain.flux(0), bl.flux(0))


@pytest.mark.parametrize("phase,m", [(0.7, 0), (0.7, 1), (-2.1, 2), (np.pi, 0)])
def test_bloch_plane_wave_follows_the_lattice_dispersion(oracle_lib, phase, m):
    """A lattice Bloch plane wave in 2D vacuum (periodic x, Bloch y) stays a plane wave whose amplitude obeys
    the Yee two-step recurrence exactly (to rounding)."""
    nx, ny = 16, 12
    kx = 2 * np.pi * 3 / nx
    ky = (phase + 2 * np.pi * m) / ny
    p = Problem(name="bloch-wave", ndim=2, n=(nx, ny, 1), bc=(PERIODIC, PERIODIC, PERIODIC), dtype="f64",
                steps=0, bloch=(0.0, phase, 0.0))
    o = oracle_lib.Oracle(p)
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    mode = np.exp(1j * (kx * X + ky * Y)).reshape(nx, ny, 1)
    o.set_field(2, mode)            # E_z
    o.set_field(8, mode)            # D_z (vacuum)
    K2 = 4 * np.sin(kx / 2) ** 2 + 4 * np.sin(ky / 2) ** 2
    f = 2.0 - DT * DT * K2
    c = [1.0 + 0j]
    for n in range(60):
        o.step(1)
        e = o.field(2)
        amp = e[0, 0, 0] / mode[0, 0, 0]
        # shape: every cell, including both wrap rows, is the same multiple of the mode
        assert np.max(np.abs(e - amp * mode)) < 1e-12 * max(1.0, abs(amp))
        c.append(amp)
    c = np.array(c)
    # e_1 = e_0 (H starts at zero), then c_{n+1} = f c_n - c_{n-1}
    assert abs(c[1] - c[0]) < 1e-14
    res = c[2:] - (f * c[1:-1] - c[:-2])
    assert np.max(np.abs(res)) < 1e-12


@pytest.mark.parametrize("which", ["lorentz_bath", "drude"])
def test_bloch_oblique_slab_transmission_lattice_tmm(oracle_lib, which):
    """Oblique incidence on a Bloch-periodic 2D grid (two cells along y, phase 2 ky): transmission of a slab
    equals the lattice transfer matrix of the stack with the transverse term, for a Lorentz-Bath slab and a
    thin Drude film.  The pulse (width 0.12) carries nothing near the cutoff 4 sin^2(w dt/2)/dt^2 =
    4 sin^2(ky/2) (w ~ 0.4): waves there run almost parallel to the absorbing layers, which do not take
    them, and their late arrival leaks into the transform (with width 0.2 the error grows with the run
    length: 2e-5 after 30 000 steps, 2e-4 after 60 000)."""
    from oracle.closed_form import chi_discrete, lattice_transmission
    ky = 0.4
    ny, nx = 2, 800
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
        o = oracle_lib.Oracle(_slab_problem(nx, ny, ms, w, ny * ky, steps, width=0.12))
        o.step(steps)
        return o.flux(0)
    T = run(mats) / run([])
    ref = lattice_transmission(w, DT, np.full(L, eps), np.tile(chi, (L, 1)), ky=ky)
    assert np.max(np.abs(T - ref)) < 1e-6
    # the transverse term matters: normal incidence differs by far more than the tolerance
    assert np.max(np.abs(ref - lattice_transmission(w, DT, np.full(L, eps), np.tile(chi, (L, 1))))) > 1e-3


def test_bloch_flux_is_that_of_the_complex_fields(oracle_lib):
    """The flux of a Bloch grid is the flux of the complex fields f = f_re + i f_im read back cell by cell:
    with E~ and H~ summed by hand from the complex plane fields of every step (E at t_{n+1/2}, H averaged
    over the two nodes beside the plane at t_{n+1}), Re sum (E~ x conj H~) . e_x equals the grid's flux.  The
    problem has no mirror symmetry along y (a patch over part of the period, a random complex source
    profile), so the flux at w and at -w differ and the sign of i in f_re + i f_im is fixed."""
    nx, ny, steps, p0 = 70, 5, 300, 52
    rs = np.random.default_rng(11)
    w = np.array([0.6, 0.9, 1.0, 1.3])
    p = Problem(name="bloch-flux", ndim=2, n=(nx, ny, 1), bc=(PML, PERIODIC, PERIODIC), pml_cells=(10, 0, 0),
                dtype="f64", steps=steps, bloch=(0.0, 1.1, 0.0))
    p.materials.append(LorentzBath(box((30, 45), (0, 2)), omega0=1.0, gamma0=0.05, eps_inf=2.0, sigma=0.3, n_bath=2,
                                   omega_j=np.array([0.9, 1.1]), gamma_j=np.full(2, 0.02), k_j=np.full(2, 0.1)))
    p.sources.append(Source(comp=2, box=box((20, 21), (0, ny)), omega_c=1.0, width=0.5,
                            profile=rs.uniform(-1, 1, ny), profile_im=rs.uniform(-1, 1, ny)))
    p.dfts.append(DftFlux(0, box((p0, p0 + 1), (0, ny)), w))
    o = oracle_lib.Oracle(p)
    ws = np.concatenate([w, -w])           # the transforms at +w and at -w
    Et = np.zeros((len(ws), ny), complex)
    Ht = np.zeros((len(ws), ny), complex)
    for n in range(steps):
        o.step(1)
        ez = o.field(2)[p0, :, 0]
        hy = 0.5 * (o.field(4)[p0 - 1, :, 0] + o.field(4)[p0, :, 0])
        Et += DT * np.exp(1j * ws[:, None] * (n + 0.5) * DT) * ez[None, :]
        Ht += DT * np.exp(1j * ws[:, None] * (n + 1.0) * DT) * hy[None, :]
    # (E x H*)_x = E_y H_z* - E_z H_y* with E_y = H_z = 0 on the 2D TM grid
    flux = -np.real(np.sum(Et * np.conj(Ht), axis=1))
    want, at_minus_w = flux[:len(w)], flux[len(w):]
    assert np.max(np.abs(o.flux(0) - want)) < 1e-12 * np.max(np.abs(want))
    # the flux at -w (what f_re - i f_im would give) differs: the check above fixes the sign of i
    assert np.max(np.abs(want - at_minus_w)) > 0.1 * np.max(np.abs(want))
