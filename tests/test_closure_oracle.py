"""Pins of the learned-closure reference (oracle/closure.py): gradients against finite
differences, the bath-force replay against the FDTD oracle's polarization update, an exact linear
closure of a one-mode bath, and training from random weights on that case."""
import numpy as np
import pytest

from fdtdb_inputs.problem import LorentzBath, Problem, PERIODIC, box
from oracle import closure as cl

DT = 0.5


def _params(width, rng, scale=0.3):
    return {k: rng.normal(0, scale, s) for k, s in cl.shapes(width).items()}


@pytest.mark.parametrize("act", ["tanh", "identity"])
def test_bptt_matches_central_differences(act):
    rng = np.random.default_rng(0)
    p = _params(8, rng)
    X = rng.normal(size=(3, 9, 3))
    Y = rng.normal(size=(3, 9))
    h0 = rng.normal(size=(3, 4)) * 0.1
    _, g = cl.loss_and_grad(p, X, Y, h0, act)
    v = cl.flatten(p)
    gv = cl.flatten(g)
    eps = 1e-6
    num = np.zeros_like(v)
    for i in range(len(v)):
        vp, vm = v.copy(), v.copy()
        vp[i] += eps
        vm[i] -= eps
        num[i] = (cl.loss(cl.unflatten(vp, 8), X, Y, h0, act) - cl.loss(cl.unflatten(vm, 8), X, Y, h0, act)) / (2 * eps)
    assert np.max(np.abs(num - gv)) / np.max(np.abs(gv)) < 1e-6


def test_bath_force_satisfies_the_polarization_update(oracle_lib):
    """Drive one Lorentz-Bath cell of the C oracle; the bath force replayed from its P sequence
    closes eq:Pz_update-LB exactly: A P^{m+1} = w0^2 dt^2 sigma E^m - (w0^2 dt^2 - 2) P^m
    - (1 - g0 dt/2 - (dt/2) sum k c) P^{m-1} - S^m."""
    wj, gj, kj = np.array([0.9, 1.0, 1.15]), np.array([0.02, 0.01, 0.03]), np.array([0.12, 0.2, 0.07])
    w0, g0, sig = 1.0, 0.01, 0.1
    p = Problem(name="0d", ndim=1, n=(1, 1, 1), bc=(PERIODIC, PERIODIC, PERIODIC), dtype="f64")
    p.materials.append(LorentzBath(box((0, 1)), omega0=w0, gamma0=g0, eps_inf=1.0, sigma=sig, n_bath=3, omega_j=wj,
                                   gamma_j=gj, k_j=kj))
    o = oracle_lib.Oracle(p)
    n = np.arange(400)
    E = np.exp(-((n - 40) / 8.0) ** 2) * np.cos(0.9 * n * DT)
    Pn = o.drive(0, 2, E)                 # P^{m+1} after E^m
    P = np.concatenate([[0.0], Pn])       # P^0 ... P^T
    S = cl.bath_force(P[None, :], DT, wj, gj, kj)[0]
    den = 1 + 0.5 * gj * DT
    skc = np.sum(kj * kj * DT / (2 * den))
    A = 1 + 0.5 * g0 * DT + 0.5 * DT * skc
    Pm1 = np.concatenate([[0.0], P[:-2]])
    lhs = A * P[1:]
    rhs = w0 ** 2 * DT ** 2 * sig * E - (w0 ** 2 * DT ** 2 - 2) * P[:-1] - (1 - 0.5 * g0 * DT - 0.5 * DT * skc) * Pm1 - S
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(lhs))
    assert np.max(np.abs(S)) > 1e-3 * np.max(np.abs(P))


def _one_mode_data(N=6, T=300, seed=3):
    """Polarization trajectories (random damped drives) and the bath force of one bath mode."""
    rng = np.random.default_rng(seed)
    w, g, k = np.array([1.05]), np.array([0.03]), np.array([0.15])
    t = np.arange(T + 1) * DT
    P = np.zeros((N, T + 1))
    for i in range(N):
        f, ph, tau = rng.uniform(0.8, 1.2), rng.uniform(0, 6.28), rng.uniform(20, 60)
        P[i] = np.sin(f * t + ph) * (1 - np.exp(-t / tau)) * np.exp(-t / (4 * tau))
    P[:, 0] = 0.0
    S = cl.bath_force(P, DT, w, g, k)
    V = np.diff(np.concatenate([np.zeros((N, 1)), P], axis=1), axis=1)[:, :T] / DT
    E = np.zeros((N, T))
    X = np.stack([E, P[:, :T], V], axis=2)
    return X, S, (w, g, k)


def test_exact_linear_closure_of_one_mode():
    """With identity activations the closure can carry (Y^{m-1}, Y^{m-2}, P^{m-1}) in its hidden
    state and reproduce the one-mode bath force exactly."""
    X, S, (w, g, k) = _one_mode_data()
    den = 1 + 0.5 * g[0] * DT
    a, b, c = (2 - w[0] ** 2 * DT ** 2) / den, -2 / den, k[0] * DT / (2 * den)
    # x = [E, P^m, V^m, h0 = Y^{m-1}, h1 = Y^{m-2}, h2 = P^{m-2}, h3]; P^{m-1} = P^m - dt V^m
    # Y^m = a Y^{m-1} + (b+1) Y^{m-2} + c (P^m - P^{m-2});  S^m = (dt/2) k (a Y^m + b Y^{m-1})
    L = np.zeros((5, 7))
    ym = np.array([0, c, 0, a, b + 1, -c, 0])                 # Y^m as a row over x
    L[0] = ym - np.eye(7)[3]                                    # h0 <- Y^m
    L[1] = np.eye(7)[3] - np.eye(7)[4]                          # h1 <- Y^{m-1}
    L[2] = np.array([0, 1, -DT, 0, 0, -1, 0])                   # h2 <- P^{m-1}
    L[4] = 0.5 * DT * k[0] * (a * ym + b * np.eye(7)[3])        # S^m
    W = 32
    p = {"W1": np.zeros((W, 7)), "b1": np.zeros(W), "W2": np.zeros((W, W)), "b2": np.zeros(W),
         "W3": np.zeros((5, W)), "b3": np.zeros(5)}
    p["W1"][:7] = np.eye(7)
    p["W2"][:7, :7] = np.eye(7)
    p["W3"][:, :7] = L
    Lval = cl.loss(p, X, S, np.zeros((X.shape[0], 4)), act="identity")
    assert Lval < 1e-28 * max(1.0, np.mean(S ** 2))
    assert np.mean(S ** 2) > 1e-6


def test_training_fits_one_mode_bath():
    """Adam from seeded random hidden layers and a zero output layer (a quiet recurrence) drives
    the one-mode linear closure's normalised loss from 1 to below 1e-3."""
    from fdtdb_inputs.philox import Stream
    X, S, _ = _one_mode_data(N=8, T=120, seed=5)
    Y = S / np.std(S)
    rs = Stream(77, 5)
    p = {k: rs.normal(int(np.prod(s))).reshape(s) * 0.3 for k, s in cl.shapes(32).items()}
    p["W3"][:] = 0.0
    p["b3"][:] = 0.0
    m, v = cl.adam_init(p)
    h0 = np.zeros((X.shape[0], 4))
    L0 = cl.loss(p, X, Y, h0, "identity")
    for it in range(1, 801):
        L, g = cl.loss_and_grad(p, X, Y, h0, "identity")
        cl.adam_step(p, g, m, v, it, lr=3e-3 * 0.995 ** it)
    L1 = cl.loss(p, X, Y, h0, "identity")
    assert L0 > 0.5 and L1 < 1e-3


def test_tbptt_one_window_is_bptt_and_windows_carry_state():
    """With one window TBPTT is plain BPTT; with several, the loss is the mean of the window losses
    of one uninterrupted forward pass (the carried state is the forward state)."""
    rng = np.random.default_rng(4)
    p = _params(8, rng)
    X = rng.normal(size=(3, 12, 3))
    Y = rng.normal(size=(3, 12))
    L1, g1 = cl.tbptt_loss_grad(p, X, Y, 12)
    L0, g0 = cl.loss_and_grad(p, X, Y, np.zeros((3, 4)))
    assert abs(L1 - L0) < 1e-15 and np.max(np.abs(cl.flatten(g1) - cl.flatten(g0))) < 1e-15
    L3, _ = cl.tbptt_loss_grad(p, X, Y, 4)
    assert abs(L3 - L0) < 1e-13 * L0          # equal-length windows: same mean squared error


def test_prepare_rebuilds_the_inputs_of_the_polarization_update(oracle_lib):
    """prepare() on the C oracle's recorded trajectory: V is the P difference entering each step,
    and the force closes eq:Pz_update-LB with the recorded E (as in the bath-force pin)."""
    wj, gj, kj = np.array([0.95, 1.1]), np.array([0.02, 0.01]), np.array([0.1, 0.15])
    w0, g0, sig = 1.0, 0.0, 0.05
    p = Problem(name="0d", ndim=1, n=(1, 1, 1), bc=(PERIODIC, PERIODIC, PERIODIC), dtype="f64")
    p.materials.append(LorentzBath(box((0, 1)), omega0=w0, gamma0=g0, eps_inf=1.0, sigma=sig, n_bath=2, omega_j=wj,
                                   gamma_j=gj, k_j=kj))
    o = oracle_lib.Oracle(p)
    n = np.arange(200)
    E = np.exp(-((n - 30) / 6.0) ** 2) * np.cos(1.0 * n * DT)
    Pn = o.drive(0, 2, E)
    X, Y, sc, S = cl.prepare(E[:, None], Pn[:, None], DT, wj, gj, kj)
    Pin = X[0, :, 1] / sc[1]
    V = X[0, :, 2] / sc[2]
    assert np.allclose(Pin[1:], Pn[:-1], rtol=0, atol=1e-15) and Pin[0] == 0.0
    assert np.allclose(V[1:] * DT, np.diff(np.concatenate([[0.0], Pn[:-1]])), rtol=0, atol=1e-15)
    skc = np.sum(kj * kj * DT / (2 * (1 + 0.5 * gj * DT)))
    A = 1 + 0.5 * g0 * DT + 0.5 * DT * skc
    Pm1 = Pin - V * DT
    rhs = (w0 ** 2 * DT ** 2 * sig * E - (w0 ** 2 * DT ** 2 - 2) * Pin - (1 - 0.5 * g0 * DT - 0.5 * DT * skc) * Pm1
           - S[0]) / A
    assert np.max(np.abs(rhs - Pn)) < 1e-14 * np.max(np.abs(Pn))
    assert abs(np.sqrt(np.mean((Y[0] / sc[3]) ** 2)) * sc[3] - 1.0) < 1e-12
