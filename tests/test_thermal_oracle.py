"""Pins of the oracle's thermal and anharmonic baths (extensions the paper names in Sec. V).

Thermal bath: every damped coordinate (P with gamma0, each Y_j with gamma_j) carries the Langevin force that
fluctuation-dissipation pairs with its damping for the effective mass rho = 1/(eps0 sigma omega0^2) of
eq:H_full, as unit-variance uniform variates from Philox4x32-10.  Anharmonic bath: a quartic term
(rho/4) lambda_j Y_j^4 in each mode's potential.  Pinned against what the mathematics and the physics fix:
  * the oracle's own Philox reproduces the published known-answer vectors and the input generator's stream;
  * lambda = 0 is the harmonic bath bit for bit; the thermal state scales as sqrt(kT) and superposes with a
    driven one (the noise enters the linear update additively);
  * an isolated damped mode is an AR(2) process whose stationary variance has a closed form, close to
    equipartition kT / (rho omega_j^2);
  * a cell with P and four coupled modes, driven by noise only, reaches the Gibbs state of eq:H_full:
    <rho omega0^2 P^2> = <rho omega_j^2 Y_j^2> = <rho Pdot^2> = <rho Ydot_j^2> = kT (the matter Hamiltonian
    is a sum of squares once (Pi_P - rho sum_j k_j Y_j)^2 / (2 rho) is completed), which fails if the bath
    noise does not reach P through the substituted Y_j^{n+1} or if P's own noise is missing;
  * an anharmonic mode at temperature kT has <Y^2> = the Boltzmann average over the quartic potential
    (quadrature), and a free anharmonic mode oscillates at the frequency that harmonic balance of the
    discrete recurrence gives, 2 (cos(Omega dt) - 1) = -dt^2 (omega^2 + 3 lambda A^2 / 4).
Statistical bars are about ten standard errors of the estimate; the discretisation shifts the discrete
statistics from the continuous ones by O((omega dt)^2), below 1 % at the frequencies used.
"""
import numpy as np
import pytest
from scipy.integrate import quad

from fdtdb_inputs.philox import philox4x32
from fdtdb_inputs.problem import PML, PERIODIC, DftFlux, LorentzBath, Problem, Source, box

DT = 0.5


def _mat_problem(n, w0, g0, wj, gj, kj, kT, sig=None, lam=None, seed=7, ndim=1):
    shape = (n, 1, 1) if ndim == 1 else (n, n, n)
    p = Problem(name="thermal", ndim=ndim, n=shape, bc=(PERIODIC, PERIODIC, PERIODIC), dtype="f64", steps=0)
    bx = box((0, n)) if ndim == 1 else box((0, n), (0, n), (0, n))
    p.materials.append(LorentzBath(bx, omega0=w0, gamma0=g0, eps_inf=1.0, sigma=1.0, sigma_cells=sig,
                                   n_bath=len(wj), omega_j=np.asarray(wj, float), gamma_j=np.asarray(gj, float),
                                   k_j=np.asarray(kj, float), kT=kT, noise_seed=seed,
                                   anharmonic=None if lam is None else np.asarray(lam, float)))
    return p


def _sample(oracle_lib, p, burn, nsamp, every, comp=2):
    """Advance the material alone (E = 0) and sample P, Y and their level differences / dt."""
    o = oracle_lib.Oracle(p)
    o.drive(0, comp, np.zeros(burn))
    P, Y, Pv, Yv = [], [], [], []
    for _ in range(nsamp):
        o.drive(0, comp, np.zeros(every))
        p0, p1 = o.polarization(0, comp, 0), o.polarization(0, comp, 1)
        y0, y1 = o.bath(0, comp, 0), o.bath(0, comp, 1)
        P.append(p0); Y.append(y0); Pv.append((p0 - p1) / DT); Yv.append((y0 - y1) / DT)
    return np.array(P), np.array(Y), np.array(Pv), np.array(Yv)


def test_oracle_philox_known_answers(oracle_lib):
    """The oracle's own Philox4x32-10: the Random123 known-answer vectors, and the same words as the input
    generator's (independently pinned) Philox on random counters and keys."""
    O = oracle_lib.Oracle
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        assert tuple(int(x) for x in O.philox(ctr, key)) == want
    rs = np.random.default_rng(2)
    for _ in range(50):
        ctr = rs.integers(0, 2 ** 32, 4, dtype=np.uint64)
        key = [int(x) for x in rs.integers(0, 2 ** 32, 2, dtype=np.uint64)]
        assert np.array_equal(O.philox(ctr.astype(np.uint32), key), philox4x32(ctr[None, :], key)[0])


def _driven(thermal_kT, with_source, lam=None, seed=7):
    n = 300
    p = Problem(name="thermal-driven", ndim=1, n=(n, 1, 1), bc=(PML, PERIODIC, PERIODIC), pml_cells=(30, 0, 0),
                dtype="f64", steps=0)
    p.materials.append(LorentzBath(box((120, 180)), omega0=1.0, gamma0=0.02, eps_inf=1.5, sigma=0.1, n_bath=4,
                                   omega_j=np.array([0.9, 0.97, 1.03, 1.1]), gamma_j=np.array([0.01, 0.02, 0.03, 0.01]),
                                   k_j=np.array([0.05, 0.08, 0.06, 0.04]), kT=thermal_kT, noise_seed=seed,
                                   anharmonic=lam))
    if with_source:
        p.sources.append(Source(comp=2, box=box((60, 61)), omega_c=1.0, width=0.3))
    p.dfts.append(DftFlux(0, box((250, 251)), np.linspace(0.8, 1.2, 5)))
    return p


def _state(o):
    return np.concatenate([o.field(2).ravel(), o.field(4).ravel(), o.polarization(0, 2, 0), o.polarization(0, 2, 1),
                           o.bath(0, 2, 0).ravel(), o.bath(0, 2, 1).ravel()])


def test_harmonic_limit_scaling_and_superposition(oracle_lib):
    """lambda = 0 (the anharmonic path with zero coefficients) is the harmonic bath bit for bit; a grid driven
    by noise only scales as sqrt(kT); noise and source superpose (the update stays linear and the noise is
    additive), and two seeds give different noise."""
    steps = 600

    def run(p):
        o = oracle_lib.Oracle(p)
        o.step(steps)
        return _state(o)
    plain = run(_driven(0.0, True))
    assert np.array_equal(run(_driven(0.0, True, lam=np.zeros(4))), plain)
    t1, t4 = run(_driven(1e-4, False)), run(_driven(4e-4, False))
    assert np.max(np.abs(t4 - 2.0 * t1)) < 1e-13 * np.max(np.abs(t4))
    both = run(_driven(1e-4, True))
    assert np.max(np.abs(both - plain - t1)) < 1e-12 * np.max(np.abs(both))
    other = run(_driven(1e-4, False, seed=8))
    assert np.max(np.abs(other - t1)) > 0.1 * np.max(np.abs(t1))


def test_isolated_mode_is_the_ar2_process(oracle_lib):
    """An uncoupled damped mode (k_j = 0) follows Y^{n+1} = a Y^n + (b + 1) Y^{n-1} + s xi: its stationary
    variance is s^2 (1 - f2) / ((1 + f2) ((1 - f2)^2 - f1^2)) with f1 = a, f2 = b + 1, s^2 = (dt^2 / den)^2
    2 gamma kT omega0^2 sigma / dt, per cell with its own sigma; the closed form is within (omega dt)^2 of
    equipartition kT sigma omega0^2 / omega_j^2.  2048 cells, 8000 steps: standard error 0.2 %."""
    n = 2048
    sig = np.random.default_rng(1).uniform(0.5, 2.0, n)
    w, g, kT, w0 = 0.3, 0.05, 2.0, 0.25
    P, Y, _, _ = _sample(oracle_lib, _mat_problem(n, w0, 0.0, [w], [g], [0.0], kT, sig), 1000, 400, 20)
    den = 1 + 0.5 * g * DT
    f1, f2 = (2 - w * w * DT * DT) / den, -(1 - 0.5 * g * DT) / den
    s2 = (DT * DT / den) ** 2 * 2 * g * kT * w0 ** 2 / DT
    var = s2 * (1 - f2) / ((1 + f2) * ((1 - f2) ** 2 - f1 ** 2))
    assert abs(np.mean(Y[:, 0, :] ** 2 / sig) / var - 1) < 0.015
    assert abs(var / (kT * w0 ** 2 / w ** 2) - 1) < (w * DT) ** 2
    assert not np.any(P)             # gamma0 = 0 and E = 0: P carries no noise of its own


def test_coupled_cell_reaches_equipartition(oracle_lib):
    """P with gamma0 and four coupled damped modes, E = 0, noise only: every coordinate and velocity of the
    matter Hamiltonian at kT (2048 cells, 12 000 steps; bar 2.5 %, standard errors 0.3-0.5 %)."""
    n, w0, g0, kT = 2048, 0.25, 0.02, 1.5
    wj, gj, kj = [0.18, 0.22, 0.27, 0.31], [0.03] * 4, [0.06, 0.08, 0.07, 0.05]
    P, Y, Pv, Yv = _sample(oracle_lib, _mat_problem(n, w0, g0, wj, gj, kj, kT), 3000, 600, 20)
    rho = 1.0 / w0 ** 2
    got = [np.mean(P ** 2) * rho * w0 ** 2, np.mean(Pv ** 2) * rho]
    got += [np.mean(Y[:, j] ** 2) * rho * wj[j] ** 2 for j in range(4)]
    got += [np.mean(Yv[:, j] ** 2) * rho for j in range(4)]
    err = np.abs(np.array(got) / kT - 1)
    assert np.max(err) < 0.025, err
    # the modes are independent at equilibrium: <Y_0 Y_3> ~ 0
    c = np.mean(Y[:, 0] * Y[:, 3]) / np.sqrt(np.mean(Y[:, 0] ** 2) * np.mean(Y[:, 3] ** 2))
    assert abs(c) < 0.03


def test_noise_is_independent_across_cells_and_components(oracle_lib):
    """3D cube, two modes: the thermal state of the three components and of neighbouring cells is
    uncorrelated (a counter that drops the component or the cell would give correlation 1)."""
    n = 10
    o = oracle_lib.Oracle(_mat_problem(n, 0.25, 0.02, [0.2, 0.3], [0.05, 0.05], [0.05, 0.05], 1.0, ndim=3))
    for _ in range(400):
        o.drive(0, 0, np.zeros(1))   # drive() advances every component of the material each call
    y = [o.bath(0, c, 0)[0] for c in range(3)]
    for a, b in ((0, 1), (0, 2), (1, 2)):
        assert abs(np.corrcoef(y[a], y[b])[0, 1]) < 0.15
    assert abs(np.corrcoef(y[0][:-1], y[0][1:])[0, 1]) < 0.15
    assert np.all(np.abs(y[0]) > 0)


def test_anharmonic_mode_follows_the_boltzmann_average(oracle_lib):
    """Uncoupled mode with the quartic term at temperature kT: <Y^2> equals the Boltzmann average over
    V = rho (omega^2 Y^2 / 2 + lambda Y^4 / 4) (quadrature) within 2 %; the harmonic value is 63 % off."""
    n, w0, w, g, kT, lam = 2048, 0.25, 0.2, 0.05, 1.0, 0.05
    rho = 1.0 / w0 ** 2
    _, Y, _, Yv = _sample(oracle_lib, _mat_problem(n, w0, 0.0, [w], [g], [0.0], kT, lam=[lam]), 1500, 500, 20)
    V = lambda y: rho * (0.5 * w * w * y * y + 0.25 * lam * y ** 4) / kT
    Z = quad(lambda y: np.exp(-V(y)), -np.inf, np.inf)[0]
    m2 = quad(lambda y: y * y * np.exp(-V(y)), -np.inf, np.inf)[0] / Z
    assert abs(np.mean(Y ** 2) / m2 - 1) < 0.02
    assert abs(np.mean(Yv ** 2) * rho / kT - 1) < 0.03     # kinetic equipartition is unchanged
    assert m2 / (kT / (rho * w * w)) < 0.5


def test_anharmonic_mode_frequency_shift(oracle_lib):
    """A free undamped quartic mode (k = gamma = kT = 0) started at rest at A = 1: its frequency from the
    zero crossings over 9000 steps equals the first-harmonic balance of the discrete recurrence,
    Omega = (2/dt) asin((dt/2) sqrt(omega^2 + 3 lambda A^2 / 4)), to 1 % of the shift it predicts
    (lambda A^2 / omega^2 = 0.004; the second-order terms are ~1e-4 of the shift)."""
    w, lam, A = 0.3, 0.00036, 1.0
    o = oracle_lib.Oracle(_mat_problem(1, 0.25, 0.0, [w], [0.0], [0.0], 0.0, lam=[lam]))
    o.set_bath(0, 2, 0, np.array([A]))
    o.set_bath(0, 2, 1, np.array([A]))
    ys = [A]
    for _ in range(9000):
        o.drive(0, 2, np.zeros(1))
        ys.append(o.bath(0, 2, 0)[0, 0])
    ys = np.array(ys)
    idx = np.where(np.sign(ys[:-1]) != np.sign(ys[1:]))[0]
    tc = idx + ys[idx] / (ys[idx] - ys[idx + 1])
    om = 2 * np.pi / (2 * np.mean(np.diff(tc)) * DT)
    amp = np.max(np.abs(ys))
    pred = 2 / DT * np.arcsin(DT / 2 * np.sqrt(w * w + 0.75 * lam * amp ** 2))
    harm = 2 / DT * np.arcsin(DT / 2 * w)
    assert abs(om - pred) < 0.01 * abs(pred - harm)


def _xi(counter_cell, n, c, v, key):
    """The documented variate: sqrt(12) (u - 1/2), u = (x + 1/2) / 2^32, x = lane v % 4 of
    Philox(counter (cell, n, c, v // 4), key), from the input generator's own Philox."""
    x = philox4x32(np.array([[counter_cell, n, c, v // 4]], np.uint64), key)[0][v % 4]
    return (((float(x) + 0.5) / 2.0 ** 32) - 0.5) * 3.4641016151377544


def test_discrete_equations_of_motion_hold_with_the_documented_noise(oracle_lib):
    """After each update of a 3D material (box inside a larger grid, per-cell sigma, thermal and anharmonic
    bath, random levels and drive), the central-difference equations of motion the scheme discretises hold
    to rounding, with the noise computed here from the documented counter (grid cell index, step, component,
    variate / 4):
      (P' - 2P + P_)/dt^2 + gamma0 (P' - P_)/(2 dt) + sum_j k_j (Y_j' - Y_j_)/(2 dt) + omega0^2 P
          = omega0^2 sigma E + eta_P,
      (Y' - 2Y + Y_)/dt^2 + gamma_j (Y' - Y_)/(2 dt) + omega_j^2 Y + lambda_j Y^3 = k_j (P' - P_)/(2 dt) + eta_j,
    eta = sqrt(2 gamma kT omega0^2 sigma / dt) xi.  A P update that leaves the noise or the quartic force out
    of the substituted Y_j^{n+1}, or a noise counter laid out otherwise, fails this."""
    rs = np.random.default_rng(4)
    n = (3, 4, 5)
    lo, hi = (1, 0, 1), (3, 4, 5)
    nc = int(np.prod(np.subtract(hi, lo)))
    w0, g0, kT, seed = 0.9, 0.03, 0.7, 0x1234567890ABCDEF
    wj, gj, kj, lam = (np.array([0.8, 1.0, 1.15]), np.array([0.02, 0.05, 0.04]), np.array([0.3, 0.2, 0.25]),
                       np.array([0.4, -0.1, 0.2]))
    sig = rs.uniform(0.3, 1.5, nc)
    p = Problem(name="eom", ndim=3, n=n, bc=(PERIODIC, PERIODIC, PERIODIC), dtype="f64", steps=0)
    p.materials.append(LorentzBath((lo, hi), omega0=w0, gamma0=g0, eps_inf=1.0, sigma_cells=sig, n_bath=3,
                                   omega_j=wj, gamma_j=gj, k_j=kj, kT=kT, noise_seed=seed, anharmonic=lam))
    o = oracle_lib.Oracle(p)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    gidx = np.array([(i * n[1] + j) * n[2] + k for i in range(lo[0], hi[0]) for j in range(lo[1], hi[1])
                     for k in range(lo[2], hi[2])])
    for c in range(3):
        for lvl in range(2):
            o.set_polarization(0, c, lvl, rs.normal(size=nc))
            o.set_bath(0, c, lvl, rs.normal(size=3 * nc))
    worst = 0.0
    for step in range(3):
        before = [(o.polarization(0, c, 0), o.polarization(0, c, 1), o.bath(0, c, 0), o.bath(0, c, 1)) for c in range(3)]
        e = rs.normal()
        o.drive(0, 2, np.array([e]))          # E_z = e in the box, E_x = E_y = 0
        for c in range(3):
            P, P_, Y, Y_ = before[c]
            Pn, Yn = o.polarization(0, c, 0), o.bath(0, c, 0)
            assert np.array_equal(o.polarization(0, c, 1), P) and np.array_equal(o.bath(0, c, 1), Y)
            E = e if c == 2 else 0.0
            etaP = np.sqrt(2 * g0 * kT * w0 ** 2 * sig / DT) * np.array([_xi(q, step, c, 3, key) for q in gidx])
            lhs = (Pn - 2 * P + P_) / DT ** 2 + g0 * (Pn - P_) / (2 * DT) + kj @ (Yn - Y_) / (2 * DT) + w0 ** 2 * P
            res = lhs - (w0 ** 2 * sig * E + etaP)
            worst = max(worst, np.max(np.abs(res)) / np.max(np.abs(lhs)))
            for jb in range(3):
                eta = np.sqrt(2 * gj[jb] * kT * w0 ** 2 * sig / DT) * np.array([_xi(q, step, c, jb, key) for q in gidx])
                lhs = (Yn[jb] - 2 * Y[jb] + Y_[jb]) / DT ** 2 + gj[jb] * (Yn[jb] - Y_[jb]) / (2 * DT) \
                    + wj[jb] ** 2 * Y[jb] + lam[jb] * Y[jb] ** 3
                res = lhs - (kj[jb] * (Pn - P_) / (2 * DT) + eta)
                worst = max(worst, np.max(np.abs(res)) / np.max(np.abs(lhs)))
    assert worst < 1e-12, worst
