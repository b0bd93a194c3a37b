"""Learned bath closure: FP64 reference of the forward pass, backpropagation through time and Adam
(TEST INFRASTRUCTURE ONLY).

The closure replaces the explicit bath of a Lorentz-Bath cell.  The bath enters the polarization
update eq:Pz_update-LB only through the force term (dt/2) sum_j k_j (a_j Y_j^n + b_j Y_j^{n-1}) and
the constant sum_j k_j c_j inside A; it is linear and driven only by the polarization history
(eq:EOM_LorentzBath-2), so a recurrent filter of that history can stand in for it.  Per cell and
component a hidden state h (K = 4) evolves as

    x_t = [E_t s_E, P_t s_P, V_t s_V, h_t]          (V = (P^{n+1/2} - P^{n-1/2}) / dt)
    z1 = act(W1 x_t + b1),  z2 = act(W2 z1 + b2),  o_t = W3 z2 + b3       (act = tanh)
    h_{t+1} = h_t + o_t[0:4],   bath force = o_t[4] / s_S.

Training (teacher forced): windows of recorded (E, P, V) with the bath force S of the explicit
bath as target; loss = mean over windows and steps of (o_t[4] - S_t s_S)^2.  Gradients by
backpropagation through time within a window (the hidden state entering a window is a
constant).  Adam (Kingma and Ba 2015) with bias correction.
"""
from __future__ import annotations

import numpy as np

NIN, K, NOUT = 7, 4, 5
PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def shapes(width: int):
    return {"W1": (width, NIN), "b1": (width,), "W2": (width, width), "b2": (width,), "W3": (NOUT, width),
            "b3": (NOUT,)}


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], np.float64).ravel() for k in PARAM_ORDER])


def unflatten(v: np.ndarray, width: int) -> dict:
    out, i = {}, 0
    for k in PARAM_ORDER:
        shp = shapes(width)[k]
        n = int(np.prod(shp))
        out[k] = np.asarray(v[i:i + n], np.float64).reshape(shp)
        i += n
    return out


def _act(a, kind):
    return np.tanh(a) if kind == "tanh" else a


def _dact(z, kind):
    return 1.0 - z * z if kind == "tanh" else np.ones_like(z)


def forward(p: dict, X: np.ndarray, h0: np.ndarray, act: str = "tanh"):
    """X: [N, T, 3] scaled inputs; h0: [N, 4].  Returns o [N, T, 5], h [N, T+1, 4], cache."""
    N, T, _ = X.shape
    h = np.zeros((N, T + 1, K))
    h[:, 0] = h0
    o = np.zeros((N, T, NOUT))
    xs, z1s, z2s = np.zeros((N, T, NIN)), np.zeros((N, T, p["W1"].shape[0])), np.zeros((N, T, p["W1"].shape[0]))
    for t in range(T):
        x = np.concatenate([X[:, t], h[:, t]], axis=1)
        z1 = _act(x @ p["W1"].T + p["b1"], act)
        z2 = _act(z1 @ p["W2"].T + p["b2"], act)
        ot = z2 @ p["W3"].T + p["b3"]
        o[:, t] = ot
        h[:, t + 1] = h[:, t] + ot[:, :K]
        xs[:, t], z1s[:, t], z2s[:, t] = x, z1, z2
    return o, h, (xs, z1s, z2s)


def loss(p: dict, X, Y, h0, act="tanh") -> float:
    """Y: [N, T] scaled targets."""
    o, _, _ = forward(p, X, h0, act)
    return float(np.mean((o[:, :, K] - Y) ** 2))


def loss_and_grad(p: dict, X, Y, h0, act="tanh"):
    """Loss and its gradient by backpropagation through time (FP64)."""
    N, T, _ = X.shape
    o, h, (xs, z1s, z2s) = forward(p, X, h0, act)
    r = o[:, :, K] - Y
    L = float(np.mean(r ** 2))
    g = {k: np.zeros_like(v) for k, v in p.items()}
    dh = np.zeros((N, K))                       # dL/dh_{t+1}
    scale = 2.0 / (N * T)
    for t in range(T - 1, -1, -1):
        do = np.concatenate([dh, (scale * r[:, t])[:, None]], axis=1)     # [N, 5]
        g["W3"] += do.T @ z2s[:, t]
        g["b3"] += do.sum(0)
        da2 = (do @ p["W3"]) * _dact(z2s[:, t], act)
        g["W2"] += da2.T @ z1s[:, t]
        g["b2"] += da2.sum(0)
        da1 = (da2 @ p["W2"]) * _dact(z1s[:, t], act)
        g["W1"] += da1.T @ xs[:, t]
        g["b1"] += da1.sum(0)
        dx = da1 @ p["W1"]
        dh = dh + dx[:, 3:]
    return L, g


def adam_init(p: dict):
    return {k: np.zeros_like(v) for k, v in p.items()}, {k: np.zeros_like(v) for k, v in p.items()}


def adam_step(p: dict, g: dict, m: dict, v: dict, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1)."""
    for k in p:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] ** 2
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


def bath_force(P: np.ndarray, dt: float, wj, gj, kj) -> np.ndarray:
    """Bath force term of eq:Pz_update-LB along polarization trajectories.

    P: [N, T+1] with P[:, m] = P at paper level m (P[:, 0] = P^{1/2} ... in grid time), starting
    from rest.  The bath follows eq:Yzj_finite_difference driven by P; the force used in the update
    producing P[:, m+1] is (dt/2) sum_j k_j (a_j Y_j^m + b_j Y_j^{m-1}).  Returns S [N, T].
    """
    N, T1 = P.shape
    T = T1 - 1
    den = 1.0 + 0.5 * np.asarray(gj) * dt
    a = (2.0 - np.asarray(wj) ** 2 * dt * dt) / den
    b = -2.0 / den
    c = np.asarray(kj) * dt / (2.0 * den)
    Y0 = np.zeros((N, len(wj)))      # Y^{m}
    Ym = np.zeros((N, len(wj)))      # Y^{m-1}
    Pm = np.zeros(N)                 # P^{m-1}
    S = np.zeros((N, T))
    for m in range(T):
        S[:, m] = 0.5 * dt * (Y0 * a + Ym * b) @ kj
        Yn = a * Y0 + (b + 1.0) * Ym + c * (P[:, m + 1] - Pm)[:, None]
        Ym, Y0 = Y0, Yn
        Pm = P[:, m]
    return S


def prepare(E: np.ndarray, P: np.ndarray, dt: float, wj, gj, kj):
    """Training inputs from a recorder's output.

    E, P: [T, N] with row n = E^{n+1/2} and the new P^{n+3/2} of step n, starting from rest.
    Returns X [N, T, 3] (scaled E, P, V at each step's input), Y [N, T] (scaled bath force),
    scales (s_E, s_P, s_V, s_S) = 1 / rms of each, and the unscaled force S [N, T].
    """
    E = np.asarray(E, np.float64).T
    Pn = np.asarray(P, np.float64).T
    N, T = E.shape
    Pfull = np.concatenate([np.zeros((N, 1)), Pn], axis=1)        # P^{1/2} = 0 ... P^{T+1/2}
    S = bath_force(Pfull, dt, wj, gj, kj)
    Pin = Pfull[:, :T]                                              # the P entering step n
    Pprev = np.concatenate([np.zeros((N, 1)), Pfull[:, :T - 1]], axis=1)
    V = (Pin - Pprev) / dt

    def inv_rms(a):
        r = np.sqrt(np.mean(a * a))
        return 1.0 / r if r > 0 else 1.0

    sc = np.array([inv_rms(E), inv_rms(Pin), inv_rms(V), inv_rms(S)])
    X = np.stack([E * sc[0], Pin * sc[1], V * sc[2]], axis=2)
    return X, S * sc[3], sc, S


def tbptt_loss_grad(p: dict, X, Y, window: int, act="tanh"):
    """Truncated BPTT over consecutive windows from step 0: the hidden state entering window c
    is the forward state at its first step (held constant); returns the mean over windows of the
    window loss and of its gradient."""
    N, T, _ = X.shape
    _, h, _ = forward(p, X, np.zeros((N, K)), act)
    nwin = T // window
    Ls, G = 0.0, {k: np.zeros_like(v) for k, v in p.items()}
    for c in range(nwin):
        sl = slice(c * window, (c + 1) * window)
        L, g = loss_and_grad(p, X[:, sl], Y[:, sl], h[:, c * window], act)
        Ls += L / nwin
        for k in G:
            G[k] += g[k] / nwin
    return Ls, G
