"""Checkpoint / resume through the C ABI: a run saved after n1 steps and resumed on a fresh grid of
the same set-up equals the uninterrupted run bitwise (fields, both polarization and bath levels,
CPML psi via the fields they feed, learned-closure state, DFT flux with unflushed staging slots at
the save, energy samples), and a state file of another set-up is refused."""
import os

import numpy as np
import pytest

from fdtdb_inputs import configs
from fdtdb_inputs.problem import PERIODIC, PML, DftFlux, EnergyMonitor, LorentzBath, Problem, Source, box

pytestmark = pytest.mark.gpu


def _crop3d():
    # the 3D planar cavity layout (CPML z layers, Drude mirrors, Lorentz-Bath N_b = 8 with per-cell
    # sigma, plane source, FP64 z-flux DFT) on a 12 x 12 crop, FP32 state
    p = configs.config2_3d(nx=12, ny=12, steps=0, nfreq=32, dtype="f32")
    p.energies.append(EnergyMonitor(box((0, 12), (0, 12), (32, 480)), every=7))
    return p


def _closure1d():
    p = Problem(name="ck-closure", ndim=1, n=(400, 1, 1), bc=(PML, PERIODIC, PERIODIC), pml_cells=(32, 0, 0),
                dtype="f32")
    p.materials.append(LorentzBath(box((150, 250)), omega0=1.0, gamma0=0.01, eps_inf=1.0, sigma=0.05, n_bath=4,
                                   omega_j=np.linspace(0.9, 1.1, 4), gamma_j=np.full(4, 0.01),
                                   k_j=np.full(4, 0.05)))
    p.sources.append(Source(comp=2, box=box((100, 101)), omega_c=1.0, width=0.5))
    p.dfts.append(DftFlux(0, box((300, 301)), np.linspace(0.5, 1.5, 64)))
    return p


def _state(g, p, closure):
    from fdtdb_inputs.problem import active_components
    e, h = active_components(p.ndim)
    out = {f"f{c}": g.field(c) for c in list(e) + list(h)}
    for mi, m in enumerate(p.materials):
        if isinstance(m, LorentzBath):
            for c in e:
                for lvl in (0, 1):
                    out[f"P{mi}{c}{lvl}"] = g.polarization(mi, c, lvl)
                    if not closure:
                        out[f"Y{mi}{c}{lvl}"] = g.bath(mi, c, lvl)
                if closure:
                    out[f"h{mi}{c}"] = g.closure_state(mi, c)
    for k in range(len(p.dfts)):
        out[f"flux{k}"] = g.flux(k)
    for k in range(len(p.energies)):
        out[f"energy{k}"] = g.energy(k)
    return out


@pytest.mark.parametrize("case", ["crop3d", "closure1d"])
@pytest.mark.parametrize("graph", [0, 16])
def test_resume_equals_uninterrupted_run(tmp_path, case, graph):
    from paper_2505_23963_amd import Grid, closure_weights
    p = _crop3d() if case == "crop3d" else _closure1d()
    closures = None
    if case == "closure1d":
        w = configs.closure_init(seed=5, hidden_scale=0.3, state_scale=0.3, force_scale=1e-3)
        closures = {0: {"weights": closure_weights(w), "scales": [1.0, 1.0, 1.0, 1.0]}}
    n1, n2 = 93, 150          # 93: odd, and not a multiple of the 64-slot DFT staging
    print(f"[gpu] checkpoint {case} graph={graph} n1={n1} n2={n2}", flush=True)
    ref = Grid(p, graph_chunk=graph, closures=closures)
    ref.step(n1 + n2)
    want = _state(ref, p, closures is not None)
    del ref
    a = Grid(p, graph_chunk=graph, closures=closures)
    a.step(n1)
    path = os.path.join(str(tmp_path), "grid.state")
    a.save_state(path)
    a.step(n2)                 # the saved grid itself keeps going unchanged
    got_a = _state(a, p, closures is not None)
    del a
    b = Grid(p, graph_chunk=graph, closures=closures)
    b.load_state(path)
    assert b.steps_done == n1
    b.step(n2)
    got_b = _state(b, p, closures is not None)
    for k, v in want.items():
        assert np.array_equal(got_a[k], v), k
        assert np.array_equal(got_b[k], v), k


def test_state_of_another_setup_is_refused(tmp_path):
    from paper_2505_23963_amd import FdtdbError, Grid
    p = _closure1d()
    a = Grid(p)
    a.step(10)
    path = os.path.join(str(tmp_path), "grid.state")
    a.save_state(path)
    q = _closure1d()
    q.sources[0] = Source(comp=2, box=box((100, 101)), omega_c=1.1, width=0.5)
    b = Grid(q)
    b.step(3)
    before = b.field(2)
    with pytest.raises(FdtdbError) as ei:
        b.load_state(path)
    assert ei.value.status == -6 and "set-up" in str(ei.value)
    assert np.array_equal(b.field(2), before) and b.steps_done == 3
    with open(path, "r+b") as f:     # a truncated file of the right set-up leaves the grid unchanged
        f.truncate(200)
    c = Grid(p)
    c.step(4)
    with pytest.raises(FdtdbError):
        c.load_state(path)
    assert c.steps_done == 4


def test_state_of_other_weights_or_sigma_is_refused(tmp_path):
    """The set-up fingerprint covers the learned closure's weights and the per-cell sigma values: a state
    saved with one set of either is refused by a grid that has another (same shapes otherwise)."""
    from paper_2505_23963_amd import FdtdbError, Grid
    from paper_2505_23963_amd.fdtdb import closure_weights
    d = configs.closure_init(3, hidden_scale=0.3, state_scale=1e-3, force_scale=0.05)
    w1 = closure_weights(d)
    w2 = w1.copy()
    w2[100] += 1e-3
    sc = (1.0, 10.0, 10.0, 100.0)
    p = _closure1d()
    a = Grid(p, closures={0: {"weights": w1, "scales": sc}})
    a.step(10)
    path = os.path.join(str(tmp_path), "closure.state")
    a.save_state(path)
    b = Grid(p, closures={0: {"weights": w2, "scales": sc}})
    with pytest.raises(FdtdbError) as ei:
        b.load_state(path)
    assert ei.value.status == -6
    Grid(p, closures={0: {"weights": w1, "scales": sc}}).load_state(path)      # same weights: accepted
    q = _crop3d()
    g = Grid(q)
    g.step(5)
    path3 = os.path.join(str(tmp_path), "crop.state")
    g.save_state(path3)
    r = _crop3d()
    r.materials[1].sigma_cells = np.array(r.materials[1].sigma_cells)
    r.materials[1].sigma_cells.flat[7] *= 1.01
    with pytest.raises(FdtdbError) as ei:
        Grid(r).load_state(path3)
    assert ei.value.status == -6
