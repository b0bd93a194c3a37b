"""GPU parity of the batched 1D cavity path (fdtdb_batch_*) against the FP64 oracle, the grid
path, and itself under different tile shapes."""
import numpy as np
import pytest

from fdtdb_inputs import configs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def cavities(n, steps, dtype, lengths=None):
    return configs.config3_cavities(ncav=n, steps=steps, dtype=dtype, nfreq=64, lengths=lengths)


@pytest.mark.parametrize("tiling", [(16, 256), (40, 256)])
def test_batch_fp64_matches_oracle(oracle_lib, tiling):
    """Four cavities of the batched workload (N_b = 32) in FP64, against the oracle run per cavity."""
    from paper_2505_23963_amd import Batch
    ps = cavities(4, 2500, "f64", lengths=[1500, 1777, 2049, 2600])
    print(f"[gpu] batch f64 tiling={tiling}", flush=True)
    b = Batch(ps, tiling=tiling)
    b.step(2500)
    b.synchronize()
    for c, p in enumerate(ps):
        o = oracle_lib.run(p, steps=2500)
        for comp in (2, 4):
            assert rel(b.field(c, comp), o.field(comp)[:, 0, 0]) < 1e-12, (c, comp)
        assert rel(b.flux(c), o.flux(0)) < 1e-11, c
        eb, eo = b.energy(c), o.energy(0)
        assert eb.shape == eo.shape
        assert np.max(np.abs(eb - eo)) < 1e-11 * np.abs(eo).max(), c


def test_batch_fp32_autotuned_matches_oracle(oracle_lib):
    from paper_2505_23963_amd import Batch
    ps = cavities(6, 3000, "f32")
    print("[gpu] batch f32 autotune", flush=True)
    b = Batch(ps)
    b.step(3000)
    b.synchronize()
    print("tiling chosen:", b.tiling, flush=True)
    for c in (0, 3, 5):
        o = oracle_lib.run(ps[c], steps=3000)
        assert rel(b.field(c, 2), o.field(2)[:, 0, 0]) < 1e-5, c
        assert rel(b.flux(c), o.flux(0)) < 1e-5, c


def test_batch_matches_grid_path():
    """The on-chip batched kernel and the HBM grid path agree on a cavity (same FP32 storage)."""
    from paper_2505_23963_amd import Batch, Grid
    ps = cavities(3, 1200, "f32", lengths=[1600, 2222, 3001])
    b = Batch(ps, tiling=(32, 512))
    b.step(1200)
    for c in range(3):
        g = Grid(ps[c])
        g.step(1200)
        assert rel(b.field(c, 2), g.field(2)[:, 0, 0]) < 1e-6, c
        assert rel(b.flux(c), g.flux(0)) < 1e-6, c


def test_batch_fields_independent_of_tile_shape():
    """Owned cells are computed with the same arithmetic whatever the tile: fields agree bitwise."""
    from paper_2505_23963_amd import Batch
    ps = cavities(5, 700, "f32")
    out = []
    for tiling in [(16, 256), (32, 512), (64, 512)]:
        b = Batch(ps, tiling=tiling)
        b.step(700)
        out.append([b.field(c, 2) for c in range(5)] + [b.field(c, 4) for c in range(5)])
    for k in range(1, 3):
        for a, c in zip(out[0], out[k]):
            assert np.array_equal(a, c)


def test_batch_full_workload_short(oracle_lib):
    """All 64 cavities of the batched workload (lengths 1500-4000, N_b = 32) for 400 steps,
    two sampled cavities checked against the oracle."""
    from paper_2505_23963_amd import Batch
    ps = configs.config3_cavities(steps=400, nfreq=512)
    b = Batch(ps)
    b.step(400)
    b.synchronize()
    for c in (7, 50):
        o = oracle_lib.run(ps[c], steps=400)
        assert rel(b.field(c, 2), o.field(2)[:, 0, 0]) < 1e-5, c


def _fit_rate(trace, every, dt, t_lo, t_hi):
    """Least-squares fit of E_bath(t) = E_inf (1 - exp(-G t)) on [t_lo, t_hi]: for each G the best E_inf is
    linear, G by a coarse scan and golden-section refinement."""
    t = np.arange(len(trace)) * every * dt
    sel = (t >= t_lo) & (t <= t_hi)
    t, y = t[sel], trace[sel]

    def resid(G):
        f = 1.0 - np.exp(-G * t)
        e = (f @ y) / (f @ f)
        return np.sum((y - e * f) ** 2)

    grid = np.geomspace(1e-5, 1.0, 400)
    k = int(np.argmin([resid(G) for G in grid]))
    a, b = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
    phi = (np.sqrt(5.0) - 1.0) / 2.0
    for _ in range(80):
        c, d = b - phi * (b - a), a + phi * (b - a)
        if resid(c) < resid(d):
            b = d
        else:
            a = c
    return 0.5 * (a + b)


def test_batch_relaxation_rates_match_oracle(oracle_lib):
    """Relaxation rates fitted to the bath-energy growth (FP32 batched path vs FP64 oracle, same fit on
    [2 t0, pi / dw], before the discrete bath revives)."""
    from paper_2505_23963_amd import Batch
    ps = cavities(4, 600, "f32", lengths=[1500, 1900, 2400, 3100])
    b = Batch(ps, tiling=(32, 512))
    b.step(600)
    b.synchronize()
    for c, p in enumerate(ps):
        o = oracle_lib.run(p, steps=600)
        eg, eo = b.energy(c)[:, 2], o.energy(0)[:, 2]
        m = p.materials[1]
        dw = 0.4 / (m.n_bath - 1)
        t0 = 5.0 / p.sources[0].width
        every = p.energies[0].every
        Gg = _fit_rate(eg, every, p.courant, 2 * t0, np.pi / dw)
        Go = _fit_rate(eo, every, p.courant, 2 * t0, np.pi / dw)
        print(f"[gpu] cavity {c}: rate {Gg:.6e} (GPU) vs {Go:.6e} (oracle)", flush=True)
        assert Go > 0 and abs(Gg - Go) <= 1e-4 * Go, (c, Gg, Go)


def test_batch_retile_after_step_zero_keeps_energy_layout():
    """A tile shape set after a zero-step call (which already sized the energy partials for the first
    shape) re-lays the energy buffer out for the new shape: the energy traces then equal those of a
    batch given that shape from the start, bit for bit."""
    from paper_2505_23963_amd import Batch
    ps = cavities(3, 300, "f32", lengths=[1500, 2300, 3100])
    a = Batch(ps, tiling=(32, 512))
    a.step(0)
    from paper_2505_23963_amd.fdtdb import lib, _bcheck
    _bcheck(lib().fdtdb_batch_set_tiling(a.h, 16, 256))      # narrower tiles: more segments per cavity
    a.step(300)
    b = Batch(ps, tiling=(16, 256))
    b.step(300)
    a.synchronize()
    b.synchronize()
    for c in range(3):
        assert np.array_equal(a.energy(c), b.energy(c)), c
        assert np.array_equal(a.field(c, 2), b.field(c, 2)), c


@pytest.mark.parametrize("dtype,tiling", [("f32", (32, 512)), ("f64", (16, 256))])
def test_batch_lds_poisoned_with_nan_changes_nothing(monkeypatch, dtype, tiling):
    """Check mode (FDTDB_POISON_LDS=1 when the batch is created): every LDS word of the on-chip kernel (the
    neighbour exchange rows, the DFT staging rows, the energy reduction slots) starts each launch as NaN.
    Fields, spectra and energy traces stay finite and bitwise equal to a normal run, so no launch reads an
    LDS word before a thread of that launch wrote it."""
    from paper_2505_23963_amd import Batch
    ps = cavities(4, 640, dtype, lengths=[1500, 1777, 2049, 2600])
    runs = []
    for poison in ("0", "1"):
        monkeypatch.setenv("FDTDB_POISON_LDS", poison)
        b = Batch(ps, tiling=tiling)
        b.step(640)
        b.synchronize()
        runs.append([(b.field(c, 2), b.field(c, 4), b.flux(c), b.energy(c)) for c in range(4)])
    for plain, poisoned in zip(*runs):
        for x, y in zip(plain, poisoned):
            assert np.all(np.isfinite(y))
            assert np.array_equal(x, y)
