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


def _exact_one_mode_closure(w, g, k, scales, eps):
    """Weights of the tanh closure that reproduces a one-mode bath to O(eps^2): the exact linear
    closure (hidden state Y^{m-1}, Y^{m-2}, P^{m-2}) written on the scaled inputs of the C oracle's
    closure branch, with every pre-activation shrunk by eps and the output layer grown by 1/eps."""
    den = 1 + 0.5 * g * DT
    a, b, c = (2 - w ** 2 * DT ** 2) / den, -2 / den, k * DT / (2 * den)
    sE, sP, sV, sS = scales
    L = np.zeros((5, 7))
    ym = np.array([0, c, 0, a, b + 1, -c, 0])
    L[0] = ym - np.eye(7)[3]
    L[1] = np.eye(7)[3] - np.eye(7)[4]
    L[2] = np.array([0, 1, -DT, 0, 0, -1, 0])
    L[4] = 0.5 * DT * k * (a * ym + b * np.eye(7)[3]) * sS
    # the rows above act on unscaled (E, P, V, h); the network sees (E sE, P sP, V sV, h)
    L = L / np.array([sE, sP, sV, 1, 1, 1, 1])[None, :]
    W = 32
    p = {"W1": np.zeros((W, 7)), "b1": np.zeros(W), "W2": np.zeros((W, W)), "b2": np.zeros(W),
         "W3": np.zeros((5, W)), "b3": np.zeros(5)}
    p["W1"][:7] = eps * np.eye(7)
    p["W2"][:7, :7] = np.eye(7)
    p["W3"][:, :7] = L / eps
    return p, float(k * k * DT / (2 * den))


def _cavity_1d(mat_kw, steps):
    from fdtdb_inputs.problem import CLOSED, Source
    p = Problem(name="cl1d", ndim=1, n=(120, 1, 1), bc=(CLOSED, PERIODIC, PERIODIC), dtype="f64", steps=steps)
    p.materials.append(LorentzBath(box((30, 100)), omega0=1.0, gamma0=0.01, eps_inf=1.0, sigma=0.1, **mat_kw))
    p.sources.append(Source(comp=2, box=box((20, 21)), omega_c=1.0, width=0.5, amplitude=0.3))
    return p


def test_c_closure_branch_carries_the_exact_one_mode_closure(oracle_lib):
    """The C oracle's learned-closure branch, given the exact linear closure of a one-mode bath carried
    into tanh by eps-scaling, advances a 1D cavity exactly as the explicit N_b = 1 bath does (to the
    O(eps^2) of tanh's cubic term), on inputs scaled by four different factors.  The bath is strong
    enough that leaving it out, or feeding the closure a velocity off by the 1/dt factor, moves E by
    more than 1e-3."""
    w, g, k = np.array([1.05]), np.array([0.03]), np.array([0.3])
    steps = 1500
    pe = _cavity_1d(dict(n_bath=1, omega_j=w, gamma_j=g, k_j=k), steps)
    oe = oracle_lib.run(pe)
    scales = (2.0, 3.0, 5.0, 7.0)
    wts, skc = _exact_one_mode_closure(w[0], g[0], k[0], scales, 1e-4)
    pc = _cavity_1d(dict(n_bath=1, omega_j=w, gamma_j=g, k_j=k), steps)
    oc = oracle_lib.run(pc, closures={0: {"weights": cl.flatten(wts), "scales": scales, "sum_kc": skc, "width": 32}})
    ref = oe.field(2)
    err = np.linalg.norm(oc.field(2) - ref) / np.linalg.norm(ref)
    assert err < 1e-6, err
    errP = np.linalg.norm(oc.polarization(0, 2, 0) - oe.polarization(0, 2, 0)) / np.linalg.norm(oe.polarization(0, 2, 0))
    assert errP < 1e-6, errP
    # the hidden state holds the lagged bath coordinate: h0 = Y^{n-1/2} of the explicit run
    assert np.max(np.abs(oc.hidden(0, 2)[:, 0] - oe.bath(0, 2, 1)[0])) < 1e-6 * np.max(np.abs(oe.bath(0, 2, 1)))
    # the bath matters at this coupling, and so does the velocity input's 1/dt
    pl = _cavity_1d(dict(n_bath=0), steps)
    assert np.linalg.norm(oracle_lib.run(pl).field(2) - ref) / np.linalg.norm(ref) > 1e-3
    wrong, _ = _exact_one_mode_closure(w[0], g[0], k[0], (2.0, 3.0, 5.0 * DT, 7.0), 1e-4)
    ow = oracle_lib.run(_cavity_1d(dict(n_bath=1, omega_j=w, gamma_j=g, k_j=k), steps),
                        closures={0: {"weights": cl.flatten(wrong), "scales": scales, "sum_kc": skc, "width": 32}})
    assert np.linalg.norm(ow.field(2) - ref) / np.linalg.norm(ref) > 1e-3


def test_c_closure_branch_matches_the_python_forward_pass(oracle_lib):
    """One cell of the C oracle's closure branch driven by a prescribed E, with random weights in
    tanh's nonlinear range: the polarization it produces closes eq:Pz_update-LB with the bath force
    o[4]/s_S of oracle/closure.forward run on the same inputs (E s_E, P^{n+1/2} s_P,
    (P^{n+1/2} - P^{n-1/2})/dt s_V), and the final hidden states agree."""
    rng = np.random.default_rng(21)
    prm = {kk: rng.normal(0, 0.4, s) for kk, s in cl.shapes(32).items()}
    prm["W3"][:4] *= 0.05
    w0, g0, sig, skc = 1.0, 0.01, 0.08, 0.004
    scales = np.array([1.5, 4.0, 6.0, 20.0])
    p = Problem(name="0d", ndim=1, n=(1, 1, 1), bc=(PERIODIC, PERIODIC, PERIODIC), dtype="f64")
    p.materials.append(LorentzBath(box((0, 1)), omega0=w0, gamma0=g0, eps_inf=1.0, sigma=sig))
    o = oracle_lib.Oracle(p, closures={0: {"weights": cl.flatten(prm), "scales": scales, "sum_kc": skc,
                                           "width": 32}})
    n = np.arange(300)
    E = np.exp(-((n - 40) / 10.0) ** 2) * np.cos(1.0 * n * DT)
    Pn = o.drive(0, 2, E)                                  # P^{m+1} after E^m
    P = np.concatenate([[0.0], Pn])                        # P^0 ... P^T
    Pprev = np.concatenate([[0.0], P[:-2]])                # P^{m-1}
    V = (P[:-1] - Pprev) / DT
    X = np.stack([E * scales[0], P[:-1] * scales[1], V * scales[2]], axis=1)[None]
    out, h, _ = cl.forward(prm, X, np.zeros((1, 4)))
    S = out[0, :, 4] / scales[3]
    A = 1 + 0.5 * g0 * DT + 0.5 * DT * skc
    rhs = (w0 ** 2 * DT ** 2 * sig * E - (w0 ** 2 * DT ** 2 - 2) * P[:-1] - (1 - 0.5 * g0 * DT - 0.5 * DT * skc) * Pprev
           - S) / A
    assert np.max(np.abs(rhs - Pn)) < 1e-12 * np.max(np.abs(Pn))
    assert np.max(np.abs(S)) > 0.1 * np.max(np.abs(Pn))
    assert np.max(np.abs(o.hidden(0, 2)[0] - h[0, -1])) < 1e-12 * max(1.0, np.max(np.abs(h)))
