"""GPU closure training (recorder, FP64 target replay, forward, BPTT, weight gradients, Adam)
against the FP64 reference in oracle/closure.py on the same records and weights.

Bars: targets and scales (FP64 on both sides, same FP32 records) <= 1e-12 relative; loss and
gradient <= 1e-4 relative (FP32 forward/backward on the GPU against FP64); the recorder's FP32 rows equal the FP64 oracle's fields rounded to FP32.
"""
import numpy as np
import pytest

from fdtdb_inputs import configs
from oracle import closure as cl

pytestmark = pytest.mark.gpu

DT = 0.5
BATH = (np.array([0.85, 0.95, 1.0, 1.07, 1.16]), np.array([0.02, 0.01, 0.03, 0.015, 0.02]),
        np.array([0.05, 0.12, 0.08, 0.1, 0.06]))


def _trainer(N, T, W, act="tanh", bath=BATH):
    from paper_2505_23963_amd import Trainer
    print(f"[gpu] trainer N={N} T={T} W={W} act={act} nb={len(bath[0])}", flush=True)
    return Trainer(N, T, W, DT, *bath, activation=act)


def _w32(d):
    return {k: np.asarray(v, np.float32).astype(np.float64) for k, v in d.items()}


def test_targets_and_scales_match_oracle():
    E, P = configs.closure_record(300, 256, seed=3)
    tr = _trainer(300, 256, 32)
    tr.load(E, P)
    X, Y, sc, S = cl.prepare(E, P, DT, *BATH)
    Sg = tr.targets().T
    assert np.max(np.abs(Sg - S)) <= 1e-12 * np.max(np.abs(S))
    assert np.max(np.abs(tr.scales() / sc - 1.0)) < 1e-12


@pytest.mark.parametrize("act", ["tanh", "identity"])
def test_loss_and_gradient_match_oracle_tbptt(act):
    from paper_2505_23963_amd import closure_weights
    N, T, W = 200, 192, 64
    E, P = configs.closure_record(N, T, seed=5)
    d = _w32(configs.closure_init(21, hidden_scale=0.3, state_scale=0.05, force_scale=0.2))
    d["b3"][:] = np.float32(0.01)
    tr = _trainer(N, T, W, act)
    tr.load(E, P)
    tr.set_weights(closure_weights(d))
    Lg, gg = tr.loss_grad()
    X, Y, sc, _ = cl.prepare(E, P, DT, *BATH)
    Lo, go = cl.tbptt_loss_grad(d, X, Y, W, act)
    go = cl.flatten(go)
    assert abs(Lg - Lo) <= 1e-5 * Lo, (Lg, Lo)
    err = np.linalg.norm(gg - go) / np.linalg.norm(go)
    print(f"[gpu] {act}: loss {Lg:.6e} vs {Lo:.6e}, gradient rel {err:.2e}", flush=True)
    assert err <= 1e-4
    # per block of parameters too (small blocks must not hide in the norm)
    off = 0
    for k in cl.PARAM_ORDER:
        n = d[k].size
        gk, ok = gg[off:off + n], go[off:off + n]
        assert np.linalg.norm(gk - ok) <= 1e-4 * max(np.linalg.norm(ok), 1e-3 * np.linalg.norm(go)), k
        off += n


def test_adam_updates_match_oracle_adam_step():
    """The GPU's Adam update (k_adam) element by element: two training epochs over a record of one window,
    each against oracle/closure.adam_step applied to the GPU's own gradient at the same weights, so that the
    comparison isolates the update (both moments, the bias corrections at t = 1 and t = 2, the FP64 master
    weights and their FP32 copy): equal to one FP32 ulp."""
    from paper_2505_23963_amd import closure_weights
    N, T = 64, 64
    E, P = configs.closure_record(N, T, seed=7)
    d = _w32(configs.closure_init(23, hidden_scale=0.3, state_scale=0.05, force_scale=0.2))
    tr = _trainer(N, T, T)
    tr.load(E, P)
    w = np.asarray(closure_weights(d), np.float32)
    tr.set_weights(w)
    p = {"w": w.astype(np.float64)}
    m, v = cl.adam_init(p)
    lr = 2e-3
    for t in (1, 2):
        _, g = tr.loss_grad()
        cl.adam_step(p, {"w": np.asarray(g, np.float64)}, m, v, t, lr=lr)
        tr.train(1, lr)
        got = tr.weights()
        want = p["w"].astype(np.float32)
        ulp = np.spacing(np.abs(want))
        bad = np.abs(got.astype(np.float64) - want) > ulp
        print(f"[gpu] adam step {t}: max |w_gpu - w_ref| = {np.max(np.abs(got - want)):.3e}, "
              f"moved {np.max(np.abs(want - w)):.3e}", flush=True)
        assert not np.any(bad), (t, np.flatnonzero(bad)[:8])
        assert np.max(np.abs(want.astype(np.float64) - w)) > 0.5 * t * lr   # the step really moved the weights


def test_training_fits_one_mode_bath_identity():
    """The linear special case: a one-mode bath is represented exactly by an identity-activation
    closure, and Adam on the GPU drives the normalised loss from about 1 to below 1e-3; the
    trained weights reproduce that loss in the FP64 reference."""
    from paper_2505_23963_amd import closure_weights
    bath = (np.array([1.05]), np.array([0.03]), np.array([0.15]))
    N, T = 64, 128
    E, P = configs.closure_record(N, T, seed=9)
    d = _w32(configs.closure_init(77, hidden_scale=0.3))
    tr = _trainer(N, T, T, "identity", bath)
    tr.load(E, P)
    tr.set_weights(closure_weights(d))
    lr = 3e-3 * 0.995 ** np.arange(800)
    losses = np.concatenate([tr.train(1, float(a)) for a in lr])
    print(f"[gpu] identity fit: loss {losses[0]:.3e} -> {losses[-1]:.3e}", flush=True)
    assert losses[0] > 0.5 and losses[-1] < 1e-3
    X, Y, _, _ = cl.prepare(E, P, DT, *bath)
    pw = cl.unflatten(tr.weights().astype(np.float64), 32)
    Lo = cl.loss(pw, X, Y, np.zeros((N, 4)), "identity")
    assert Lo < 1.5e-3


def test_probe_records_match_oracle(oracle_lib):
    from paper_2505_23963_amd import Grid
    p = configs.config1_1d(nb=16)
    cells = np.array([0, 3, 10, 11, 25, 40, 120])           # LB box starts at x = 124; source at 134
    steps = 240
    print(f"[gpu] probe {p.name} steps={steps}", flush=True)
    g = Grid(p)
    pid = g.add_probe(1, 2, cells, steps)
    g.step(steps + 10)                                      # rows beyond the capacity are not written
    E, P = g.probe_data(pid)
    o = oracle_lib.Oracle(p)
    Eo = np.zeros((steps, len(cells)))
    Po = np.zeros((steps, len(cells)))
    for n in range(steps):
        o.step(1)
        Eo[n] = o.field(2).ravel()[124 + cells]
        Po[n] = o.polarization(1, 2).ravel()[cells]
    assert np.max(np.abs(Po)) > 1e-6
    for got, ref in ((E, Eo), (P, Po)):
        assert np.max(np.abs(got - ref.astype(np.float32))) <= 1e-6 * np.max(np.abs(ref))


def test_record_and_train_small_2d():
    """The pipeline end to end on a small 2D patch: explicit run with a recorder, FP64 targets,
    training in the linear regime (identity activations) and the carry-over into tanh; the loss
    ends far below its starting value and the tanh network keeps it."""
    from paper_2505_23963_amd import Grid, Trainer, closure_weights
    from fdtdb_inputs.philox import Stream
    # N_b = 64: the bath's revival time 2 pi / dw (about 1980 steps) lies beyond the record, so a
    # K = 4 closure can fit it (a 16-mode bath revives within 512 steps, which K = 4 cannot follow)
    p = configs.config4_2d(n=192, patch=(48, 144), nb=64, dtype="f32", src_x=40, flux_x=160)
    m = p.materials[0]
    ncell = 96 * 96
    cells = np.unique(Stream(1004, 5).integers(2400, 0, ncell - 1))[:2048]
    T = 512
    print(f"[gpu] record {len(cells)} x {T}", flush=True)
    g = Grid(p)
    pid = g.add_probe(0, 2, cells, T)
    g.step(T)
    E, P = g.probe_data(pid)
    from paper_2505_23963_amd import bath_params
    wj, gj, kj = bath_params(m.form, m.omega0, m.gamma0, m.n_bath, m.width, m.bath_gamma, m.dephasing)
    tr = Trainer(len(cells), T, 64, p.courant, wj, gj, kj, activation="identity")
    tr.load(E, P)
    tr.set_weights(closure_weights(configs.closure_init(5)))
    lin = tr.train(600, 1e-2, 0.99)
    Lid, _ = tr.loss_grad()
    tr.set_activation("tanh", 1e-4)
    L0, _ = tr.loss_grad()
    print(f"[gpu] 2d pipeline: identity {lin[0]:.3e} -> {Lid:.3e}; as tanh {L0:.3e}", flush=True)
    assert np.all(np.isfinite(lin))
    assert Lid < 1e-2 * lin[0]
    assert abs(L0 - Lid) <= 0.05 * Lid
