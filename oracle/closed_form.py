"""Closed forms for pinning the FDTD-Bath oracle (TEST INFRASTRUCTURE ONLY).

Units: c = eps0 = 1, dx = 1, angular frequencies.  Time dependence exp(-i w t)
as in the paper's Fourier transforms (Sec. II.A-B), so a DFT with kernel
exp(+i w t) turns d/dt into -i w.
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------------ Table 1 (Sec. III)
def table1_bath(form: str, omega0: float, gamma0: float, nb: int, width: float, bath_gamma: float,
                dephasing: float):
    """Bath parameters of the 'uniform' / 'lorentzian' / 'gaussian' forms (Table 1 and its footnote).

    Frequencies evenly spaced on [omega0 - width/2, omega0 + width/2], one
    damping bath_gamma for all, k_b = sqrt(2 dw dephasing / pi) with
    dw = width / (nb - 1) (eq:bath_dephasing_value_uniform), and for the
    non-uniform forms k_j^2 modulated by a Lorentzian / Gaussian of linewidth
    Gamma = gamma0 + dephasing.
    """
    w = np.array([omega0 - width / 2 + width * j / (nb - 1) for j in range(nb)], dtype=np.float64)
    dw = width / (nb - 1)
    kb = np.sqrt(2.0 * dw / np.pi * dephasing)
    G = gamma0 + dephasing
    if form == "uniform":
        k = np.full(nb, kb)
    elif form == "lorentzian":
        k = kb * np.sqrt(G ** 2 / (G ** 2 + (w - omega0) ** 2))
    elif form == "gaussian":
        k = kb * np.exp(-(w - omega0) ** 2 / (4.0 * G ** 2))
    else:
        raise ValueError(form)
    return w, np.full(nb, float(bath_gamma)), k


# ------------------------------------------------------------------ continuum susceptibilities (Sec. II)
def chi_lorentz(w, omega0, gamma, sigma):
    """eq:chi_L."""
    w = np.asarray(w, dtype=np.complex128)
    return omega0 ** 2 * sigma / (omega0 ** 2 - w ** 2 - 1j * gamma * w)


def self_energy(w, wj, gj, kj):
    """eq:chi_LB_self_energy: Sigma(w) = sum_j k_j^2 w^2 / (w_j^2 - w^2 - i g_j w)."""
    w = np.asarray(w, dtype=np.complex128)[..., None]
    return np.sum(kj ** 2 * w ** 2 / (wj ** 2 - w ** 2 - 1j * gj * w), axis=-1)


def chi_lorentz_bath(w, omega0, gamma0, sigma, wj, gj, kj):
    """eq:chi_LB."""
    w = np.asarray(w, dtype=np.complex128)
    return omega0 ** 2 * sigma / (omega0 ** 2 - w ** 2 - 1j * gamma0 * w - self_energy(w, wj, gj, kj))


def gamma_lb(w, gamma0, wj, gj, kj):
    """eq:gamma_LB: gamma0 + Im Sigma / w."""
    return gamma0 + np.imag(self_energy(w, wj, gj, kj)) / np.asarray(w)


def omega_lb_sq(w, omega0, wj, gj, kj):
    """eq:omega_LB: omega0^2 - Re Sigma."""
    return omega0 ** 2 - np.real(self_energy(w, wj, gj, kj))


# ------------------------------------------------------------------ discrete (lattice) symbols
def s2(w, dt):
    """Symbol of the centred second difference: (2/dt)^2 sin^2(w dt / 2)."""
    return (2.0 / dt * np.sin(np.asarray(w) * dt / 2.0)) ** 2


def s1(w, dt):
    """Symbol of the centred first difference: sin(w dt) / dt."""
    return np.sin(np.asarray(w) * dt) / dt


def chi_discrete(w, dt, omega0, gamma0, sigma, wj=None, gj=None, kj=None, drude=False):
    """Susceptibility of the three-level recurrences at frequency w.

    Substituting X^n = X exp(-i w n dt) in the central-difference forms of
    eq:finite-difference-scheme turns the second difference into -s2 and the
    first into -i s1; eliminating the bath with eq:EOM_LorentzBath-2 gives
    chi = w0^2 sigma / (w0^2 - s2 - i g0 s1 - s1^2 sum_j k_j^2 / (w_j^2 - s2 - i g_j s1)).
    For Drude, pass omega0 = omega_p, sigma = 1 and drude=True (no restoring term).
    """
    w = np.asarray(w, dtype=np.float64)
    S2, S1 = s2(w, dt), s1(w, dt)
    restore = 0.0 if drude else omega0 ** 2
    den = restore - S2 - 1j * gamma0 * S1
    if wj is not None and len(wj):
        den = den - (S1 ** 2) * np.sum(kj ** 2 / (wj ** 2 - S2[..., None] - 1j * gj * S1[..., None]), axis=-1)
    return omega0 ** 2 * sigma / den


def chi_multipole_discrete(w, dt, kinds, omega, gamma, sigma):
    """Susceptibility of a sum of Lorentz and Drude terms advanced by their three-level recurrences: the
    terms are independent oscillators driven by the same E, so the sum of their discrete symbols."""
    out = 0.0
    for k, wp, gp, sp in zip(kinds, omega, gamma, sigma):
        out = out + (chi_discrete(w, dt, wp, gp, 1.0, drude=True) if k == "drude" else chi_discrete(w, dt, wp, gp, sp))
    return out


def multipole_margin(dt, ndim, eps_inf, kinds, omega, sigma):
    """Left side of the lossless stability condition of a sum of terms (>= 0: stable).  On the lattice a
    mode K^2 has frequencies X = s^2 solving X (eps_inf + sum_p chi_p(X)) = K^2 with chi_p = w_p^2 sigma_p /
    (w_p^2 - X) (Drude: -w_p^2 / X); with every w_p^2 < 4/dt^2 the largest root lies on the branch above all
    resonances, where the left side increases, so it stays below 4/dt^2 exactly when the left side at
    X = 4/dt^2 is at least K2max = 4 ndim.  One Lorentz term gives back lossless_margin up to a positive
    factor."""
    X = 4.0 / dt ** 2
    e = eps_inf
    for k, wp, sp in zip(kinds, omega, sigma):
        e += -wp ** 2 / X if k == "drude" else wp ** 2 * sp / (wp ** 2 - X)
    return X * e - 4.0 * ndim


def lattice_k(w, dt):
    """Vacuum lattice wavenumber: sin(k/2) = sin(w dt/2) / dt (dx = 1, Courant = dt)."""
    return 2.0 * np.arcsin(np.sin(np.asarray(w) * dt / 2.0) / dt)


def group_velocity(w, dt):
    """d w / d k of the vacuum lattice dispersion: cos(k/2) / cos(w dt / 2)."""
    k = lattice_k(w, dt)
    return np.cos(k / 2.0) / np.cos(np.asarray(w) * dt / 2.0)


def phase_velocity(w, dt):
    return np.asarray(w) / lattice_k(w, dt)


def lattice_transmission(w, dt, eps_cells, chi_cells, ky: float = 0.0):
    """|t|^2 of a 1D layer stack on the Yee lattice, vacuum on both sides.

    The lattice Helmholtz equation E_{j+1} - 2E_j + E_{j-1} + s2 (eps_j + chi_j) E_j = 0
    is integrated from a pure transmitted wave exp(i k j) behind the stack back
    to the front, where the field splits into incident and reflected lattice
    plane waves.  eps_cells: (L,) background; chi_cells: (L, nw) complex.

    ky != 0: the 2D TM lattice (E_z) with every field proportional to exp(i ky y) (oblique incidence
    on a Bloch-periodic grid): the y second difference contributes -4 sin^2(ky/2) E_j, so s2 (eps + chi)
    becomes s2 (eps + chi) - 4 sin^2(ky/2) and the vacuum wavenumber along x solves
    4 sin^2(k/2) = s2 - 4 sin^2(ky/2).
    """
    w = np.atleast_1d(np.asarray(w, dtype=np.float64))
    L = len(eps_cells)
    k = lattice_k(w, dt)
    S2 = s2(w, dt)
    if ky != 0.0:
        ty = 4.0 * np.sin(ky / 2.0) ** 2
        k = 2.0 * np.arcsin(np.sqrt(S2 - ty) / 2.0)
        eps_cells = np.asarray(eps_cells, dtype=np.float64)
        # s2 (eps + chi) - ty = s2 (eps + chi - ty / s2): fold the transverse term into chi
        chi_cells = np.asarray(chi_cells, dtype=np.complex128) - ty / S2
        S2v = S2 - ty
    else:
        S2v = S2
    # cells L, L+1 are vacuum, carrying exp(i k j)
    e_next = np.exp(1j * k * (L + 1))
    e_cur = np.exp(1j * k * L)
    # the field grows through an absorbing stack; both values are rescaled together (a linear
    # recurrence) and the scale kept as a logarithm
    logscale = np.zeros(len(w))
    for j in range(L - 1, -3, -1):
        # recurrence at node j+1 gives E_j from E_{j+1}, E_{j+2}
        node = j + 1
        if 0 <= node < L:
            fac = 2.0 - S2 * (eps_cells[node] + chi_cells[node])
        else:
            fac = 2.0 - S2v
        e_prev = fac * e_cur - e_next
        e_next, e_cur = e_cur, e_prev
        big = np.maximum(np.abs(e_cur), np.abs(e_next))
        r = np.where(big > 1e100, big, 1.0)
        e_cur, e_next = e_cur / r, e_next / r
        logscale += np.log(r)
    # now e_cur = E_{-2}, e_next = E_{-1}; E_j = A exp(ikj) + B exp(-ikj)
    jm2, jm1 = -2, -1
    det = np.exp(1j * k * jm2) * np.exp(-1j * k * jm1) - np.exp(-1j * k * jm2) * np.exp(1j * k * jm1)
    A = (e_cur * np.exp(-1j * k * jm1) - e_next * np.exp(-1j * k * jm2)) / det
    return np.exp(-2.0 * (np.log(np.abs(A)) + logscale))


# ------------------------------------------------------------------ closed-box modes and Rabi roots
def closed_box_K2(N: int):
    """Eigenvalues K_m^2 of the lattice curl-curl on N nodes with H(-1/2) = 0, E(N) = 0.

    Modes E_j = cos(k (j + 1/2)) with k (N + 1/2) = (m - 1/2) pi, K^2 = 4 sin^2(k/2).
    """
    m = np.arange(1, N + 1)
    k = (2 * m - 1) * np.pi / (2 * N + 1)
    return 4.0 * np.sin(k / 2.0) ** 2


def rabi_lattice_omegas(K2, dt, omega0, sigma, eps_inf=1.0):
    """Both polariton frequencies of a mode K^2 in a filled lossless Lorentz medium.

    Roots of eps s^4 - s^2 (eps w0^2 + w0^2 sigma + K^2) + K^2 w0^2 = 0 in X = s^2,
    mapped back by w = (2/dt) arcsin(s dt / 2).
    """
    a = eps_inf
    b = -(eps_inf * omega0 ** 2 + omega0 ** 2 * sigma + K2)
    c = K2 * omega0 ** 2
    disc = np.sqrt(b * b - 4 * a * c)
    X = np.stack([(-b - disc) / (2 * a), (-b + disc) / (2 * a)])
    return 2.0 / dt * np.arcsin(np.sqrt(X) * dt / 2.0)


def rabi_continuum(K2, omega0, sigma, eps_inf=1.0):
    """Continuum polariton pair (dt -> 0): roots of eps w^4 - w^2 (eps w0^2 + w0^2 sigma + K^2) + K^2 w0^2."""
    a = eps_inf
    b = -(eps_inf * omega0 ** 2 + omega0 ** 2 * sigma + K2)
    c = K2 * omega0 ** 2
    disc = np.sqrt(b * b - 4 * a * c)
    return np.sqrt(np.stack([(-b - disc) / (2 * a), (-b + disc) / (2 * a)]))


# ------------------------------------------------------------------ stability
def lossless_margin(dt, ndim, eps_inf, omega0=0.0, sigma=0.0, drude_wp=None):
    """Left side of the explicit-scheme stability condition (>= 0: stable).

    With X = s^2 <= 4/dt^2 required for every lattice mode, the larger root of the
    dispersion quadratic must not pass 4/dt^2:
      eps (4/dt^2 - w0^2) - w0^2 sigma - K2max (1 - w0^2 dt^2 / 4) >= 0,  K2max = 4 ndim.
    Drude: eps 4/dt^2 - w_p^2 - K2max >= 0.
    """
    K2 = 4.0 * ndim
    if drude_wp is not None:
        return eps_inf * 4.0 / dt ** 2 - drude_wp ** 2 - K2
    return eps_inf * (4.0 / dt ** 2 - omega0 ** 2) - omega0 ** 2 * sigma - K2 * (1.0 - omega0 ** 2 * dt ** 2 / 4.0)


# ------------------------------------------------------------------ bath-dephasing consistency (Sec. III)
def lorentzian_bath_im_I_approx(w, omega0, Gamma, gamma_b):
    """Approximate Im I(w) for the Lorentzian bath: (pi w / 2) G (G + gb/2) / ((w - w0)^2 + (G + gb/2)^2)."""
    G2 = Gamma + gamma_b / 2.0
    return np.pi * w / 2.0 * Gamma * G2 / ((w - omega0) ** 2 + G2 ** 2)


def gamma_polariton(Xc2, gamma_c, Xm2, gamma_m):
    """eq:gamma_polariton."""
    return Xc2 * gamma_c + Xm2 * gamma_m


# ------------------------------------------------------------------ the source (Appendix, simulation details)
def gaussian_pulse_spectrum(w, omega_c, width, amplitude=1.0):
    """Fourier transform int J(t) exp(+i w t) dt of the soft Gaussian current
    J(t) = A exp(-(t - t0)^2 / (2 tau^2)) cos(w_c (t - t0)), tau = 1/width, t0 = 5 tau, over all t:
    A exp(i w t0) tau sqrt(2 pi) / 2 [exp(-tau^2 (w - w_c)^2 / 2) + exp(-tau^2 (w + w_c)^2 / 2)].
    The source is switched off outside [0, 2 t0], where the envelope is below exp(-12.5) of its peak,
    so a sampled run differs from this by about 1e-6 of the peak."""
    w = np.asarray(w, dtype=np.float64)
    tau = 1.0 / width
    t0 = 5.0 * tau
    g = np.exp(-tau ** 2 * (w - omega_c) ** 2 / 2.0) + np.exp(-tau ** 2 * (w + omega_c) ** 2 / 2.0)
    return amplitude * np.exp(1j * w * t0) * tau * np.sqrt(2.0 * np.pi) / 2.0 * g


def point_source_response_1d(w, dt, distance):
    """E~ at `distance` nodes from a soft current J on one E node of the 1D vacuum Yee lattice, per
    unit J~ (DFT kernel exp(+i w t), E sampled at t_{n+1/2}, J at t_n, dx = 1).

    Taking the second time difference of the D line of eq:FDTD-1D and inserting the H line gives
    E_{j+1} - 2E_j + E_{j-1} + s^2 E_j = -i s J~ delta_{j,src} with s = (2/dt) sin(w dt/2); the
    outgoing solution is E~_j = -s J~ exp(i k |j - src|) / (2 sin k), sin(k/2) = s/2."""
    w = np.asarray(w, dtype=np.float64)
    k = lattice_k(w, dt)
    s = np.sqrt(s2(w, dt))
    return -s * np.exp(1j * k * abs(distance)) / (2.0 * np.sin(k))


def lattice_transmission_uniform(w, dt, eps, chi, L: int):
    """|t|^2 of one uniform layer of L cells (background eps, susceptibility chi(w)) on the 1D Yee
    lattice, vacuum on both sides: the same stack as lattice_transmission with the L identical layer
    steps of its recurrence taken at once.  The step matrix [[f, -1], [1, 0]], f = 2 - s2 (eps + chi),
    raised to the L-th power is [[U_L, -U_{L-1}], [U_{L-1}, -U_{L-2}]] with the Chebyshev polynomials
    U_n(cos q) = sin((n+1) q) / sin q at cos q = f / 2; every sine is taken relative to
    exp((L+1) |Im q|) and that scale is restored in the logarithm, so thick absorbing layers do not
    overflow."""
    w = np.atleast_1d(np.asarray(w, dtype=np.float64))
    k = lattice_k(w, dt)
    S2 = s2(w, dt)
    f = 2.0 - S2 * (eps + np.asarray(chi, dtype=np.complex128))
    q = np.arccos(f / 2.0 + 0j)
    big = (L + 1) * np.abs(q.imag)

    def U(n):       # U_n(cos q) exp(-big)
        a = 1j * (n + 1) * q
        return (np.exp(a - big) - np.exp(-a - big)) / (2j * np.sin(q))

    uL, uL1, uL2 = U(L), U(L - 1), U(L - 2)
    fv = 2.0 - S2
    # start (E_L, E_{L+1}) on the transmitted side, one vacuum step (node L), the layer, one vacuum step
    e_cur, e_next = np.exp(1j * k * L), np.exp(1j * k * (L + 1))
    e_cur, e_next = fv * e_cur - e_next, e_cur
    e_cur, e_next = uL * e_cur - uL1 * e_next, uL1 * e_cur - uL2 * e_next
    e_cur, e_next = fv * e_cur - e_next, e_cur
    jm2, jm1 = -2, -1
    det = np.exp(1j * k * jm2) * np.exp(-1j * k * jm1) - np.exp(-1j * k * jm2) * np.exp(1j * k * jm1)
    A = (e_cur * np.exp(-1j * k * jm1) - e_next * np.exp(-1j * k * jm2)) / det
    return np.exp(-2.0 * (np.log(np.abs(A)) + big))


# ------------------------------------------------------------------ what a 4-state linear closure can reach
def k4_closure_susceptibility(x, w, dt, omega0, gamma0, sigma):
    """Susceptibility of a Lorentz medium whose bath force comes from a linear recurrent filter with four
    states, driven by P and E (the learned closure with identity activations, or any such filter):
    S = G_P(z) P + G_E(z) E with G_P, G_E sharing two complex-conjugate pole pairs p_m (|p_m| < 1) and
    carrying short direct terms, z = exp(i w dt) (a causal response r p^n has the transform
    r / (1 - p z)).  In the symbols of chi_discrete this reads
        chi = w0^2 sigma (1 + C(w)) / (w0^2 - s2 - i g0 s1 + B(w)),
        B = d0 + d1 z + d2 z^2 + sum_m [b_m / (1 - p_m z) + conj],  C = e0 + e1 z + sum_m [c_m / (1 - p_m z) + conj].
    The direct terms cover every input the closure sees (E^n, P^n, P^{n-1}) with one to spare, so the
    class holds every 4-state linear closure.  x: 17 reals (|p_1|, arg p_1, |p_2|, arg p_2, b_1, b_2
    (complex, 4 reals), d0, d1, d2, c_1, c_2 (4 reals), e0, e1)."""
    w = np.asarray(w, dtype=np.float64)
    z = np.exp(1j * w * dt)
    p = [x[0] * np.exp(1j * x[1]), x[2] * np.exp(1j * x[3])]
    b = [x[4] + 1j * x[5], x[6] + 1j * x[7]]
    c = [x[11] + 1j * x[12], x[13] + 1j * x[14]]
    B = x[8] + x[9] * z + x[10] * z * z
    Cc = x[15] + x[16] * z
    for m in range(2):
        B = B + b[m] / (1 - p[m] * z) + np.conj(b[m]) / (1 - np.conj(p[m]) * z)
        Cc = Cc + c[m] / (1 - p[m] * z) + np.conj(c[m]) / (1 - np.conj(p[m]) * z)
    return omega0 ** 2 * sigma * (1 + Cc) / (omega0 ** 2 - s2(w, dt) - 1j * gamma0 * s1(w, dt) + B)


def k4_closure_best_error(w, dt, omega0, gamma0, sigma, wj, gj, kj, L, starts=6, seed=0):
    """Smallest spectral error max_w |T_4 - T| / max_w T found for 4-state linear closures on the
    transmission T of a uniform layer of L cells of the Lorentz-Bath medium (the bath of eq:chi_LB in
    its discrete form, chi_discrete) against the same layer with the closure's susceptibility.  Local
    least squares from `starts` seeded starting points: first the bath term B alone against the
    explicit bath's (a pseudomode fit), then every parameter against T itself.  Returns (error, x)."""
    from scipy.optimize import least_squares
    w = np.asarray(w, dtype=np.float64)
    T = lattice_transmission_uniform(w, dt, 1.0, chi_discrete(w, dt, omega0, gamma0, sigma, wj, gj, kj), L)
    S2, S1 = s2(w, dt), s1(w, dt)
    B_ex = -(S1 ** 2) * np.sum(kj ** 2 / (wj ** 2 - S2[:, None] - 1j * gj * S1[:, None]), axis=1)
    lo = np.array([0, -np.pi, 0, -np.pi] + [-10] * 13, dtype=np.float64)
    hi = np.array([0.99999, np.pi, 0.99999, np.pi] + [10] * 13, dtype=np.float64)

    def B_of(x):
        z = np.exp(1j * w * dt)
        out = x[8] + x[9] * z + x[10] * z * z
        for m in range(2):
            pm = x[2 * m] * np.exp(1j * x[2 * m + 1])
            bm = x[4 + 2 * m] + 1j * x[5 + 2 * m]
            out = out + bm / (1 - pm * z) + np.conj(bm) / (1 - np.conj(pm) * z)
        return out

    def T_of(x):
        return lattice_transmission_uniform(w, dt, 1.0, k4_closure_susceptibility(x, w, dt, omega0, gamma0, sigma), L)

    rng = np.random.default_rng(seed)
    best = (np.inf, None)
    for _ in range(starts):
        x0 = np.zeros(17)
        x0[0], x0[1] = np.exp(-rng.uniform(0.005, 0.1) * dt), rng.uniform(0.9, 1.1) * omega0 * dt
        x0[2], x0[3] = np.exp(-rng.uniform(0.05, 0.5) * dt), rng.uniform(0.8, 1.2) * omega0 * dt
        x0[4:8] = rng.normal(0, 1e-3, 4)
        r1 = least_squares(lambda x: np.concatenate([(B_of(x) - B_ex).real, (B_of(x) - B_ex).imag]), x0,
                           bounds=(lo, hi), max_nfev=400)
        r2 = least_squares(lambda x: T_of(x) - T, r1.x, bounds=(lo, hi), max_nfev=400)
        err = float(np.max(np.abs(T_of(r2.x) - T)) / np.max(T))
        if err < best[0]:
            best = (err, r2.x)
    return best
