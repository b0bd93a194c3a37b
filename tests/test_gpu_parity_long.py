"""FP32 parity at each workload's own length: the HIP path with FP32 state against the FP64 oracle
over the full number of steps of the 1D Fabry-Perot (20 000), 3D planar-cavity (5000), batched
cavities (50 000), 2D learned-closure workload with its explicit bath (10 000) and large 3D (4000)
workloads, on crops the oracle runs in seconds to a minute (its cell loops use every host core), and the
planar cavity at full size for 200 steps against stored oracle samples.

Measure (tests/parity_util.py): every field (E, H, each Lorentz-Bath material's P and Y) and each of
its components at every checkpoint, against the largest norm the oracle's field had so far; <= 1e-5.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from fdtdb_inputs import configs
from tests.parity_util import TOL_F32, Lockstep, flux_errors

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _lockstep(oracle_lib, p, total, every):
    from paper_2505_23963_amd import Grid
    print(f"[gpu] {p.name} n={p.n} f32, {total} steps (checkpoint every {every})", flush=True)
    g = Grid(p, dtype="f32")
    o = oracle_lib.Oracle(p)
    ls = Lockstep(g, o, p).run(total, every)
    ls.report()
    return ls, g, o


def _assert_fields(ls):
    e, c = ls.worst()
    assert e < TOL_F32 and c < TOL_F32, (e, c)


def test_fp32_config4_crop_10000_steps(oracle_lib):
    """2D TM grid, CPML on every side, Lorentzian-form bath patch of N_b = 64: 256^2 with a 128^2 patch,
    all 10 000 steps of the workload."""
    p = configs.config4_2d(n=256, patch=(64, 192), steps=10000, nfreq=64, src_x=40, flux_x=216)
    ls, g, o = _lockstep(oracle_lib, p, 10000, 2500)
    _assert_fields(ls)
    rel, _ = flux_errors(g.flux(0), o.flux(0), o.flux(0, raw=True)[1])
    print(f"  flux rel-L2 {rel:.3e}", flush=True)
    assert rel < TOL_F32


def test_fp32_config2_crop_5000_steps(oracle_lib):
    """3D planar cavity (per-cell sigma, N_b = 8, Drude mirrors, CPML), 16 x 16 x 512 crop, all 5000 steps."""
    p = configs.config2_3d(nx=16, ny=16, steps=5000, nfreq=64)
    ls, g, o = _lockstep(oracle_lib, p, 5000, 1000)
    _assert_fields(ls)
    rel, _ = flux_errors(g.flux(0), o.flux(0), o.flux(0, raw=True)[1])
    print(f"  flux rel-L2 {rel:.3e}", flush=True)
    assert rel < TOL_F32


def test_fp32_config5_crop_4000_steps(oracle_lib):
    """Large 3D layout (205-cell Lorentz-Bath slab, N_b = 16 on the component-split kernel, Gaussian-profile
    plane source), 32 x 32 x 512 crop, all 4000 steps."""
    p = configs.config5_3d_large(nx=32, ny=32, steps=4000, nfreq=32)
    ls, g, o = _lockstep(oracle_lib, p, 4000, 1000)
    _assert_fields(ls)
    rel, _ = flux_errors(g.flux(0), o.flux(0), o.flux(0, raw=True)[1])
    print(f"  flux rel-L2 {rel:.3e}", flush=True)
    assert rel < TOL_F32


def test_fp32_config5_full_planes_600_steps(oracle_lib):
    """Large 3D layout with full 512 x 512 x-planes (4 of them, periodic in x), so that the z-vector E and
    H kernels and the component-split bath kernel run with the row count, block order and neighbour
    offsets of the full grid (x-planes of 62, 224 and 410 blocks).  600 steps carry the pulse through the
    bath layer's front."""
    p = configs.config5_3d_large(nx=4, ny=512, steps=600, nfreq=16)
    ls, g, o = _lockstep(oracle_lib, p, 600, 200)
    _assert_fields(ls)
    rel, _ = flux_errors(g.flux(0), o.flux(0), o.flux(0, raw=True)[1])
    print(f"  flux rel-L2 {rel:.3e}", flush=True)
    assert rel < TOL_F32


def test_fp32_config1_20000_steps(oracle_lib):
    """The 1D Fabry-Perot workload (N_b = 16) with FP32 state for all 20 000 steps.  The in-cavity flux
    is measured against its cancellation scale; the monitor behind the opaque mirror reads FP32 rounding
    noise of the in-cavity field (|t|^2 ~ 1e-78) and is bounded by the in-cavity flux."""
    p = configs.config1_1d(steps=20000, dtype="f32")
    ls, g, o = _lockstep(oracle_lib, p, 20000, 5000)
    _assert_fields(ls)
    rel, canc = flux_errors(g.flux(0), o.flux(0), o.flux(0, raw=True)[1])
    print(f"  in-cavity flux rel-L2 {rel:.3e}, against its cancellation scale {canc:.3e}", flush=True)
    assert canc < TOL_F32
    assert np.max(np.abs(g.flux(1) - o.flux(1))) < TOL_F32 * np.max(np.abs(o.flux(0)))


def test_fp32_config3_cavities_50000_steps(oracle_lib):
    """All 64 batched cavities (N_b = 32, lengths 1500-4000) for the full 50 000 steps in the on-chip
    batched launch; four cavities spanning the sigma range checked against the oracle: E and H, the
    bath-energy trace behind the relaxation rates, and the flux against its cancellation scale."""
    from paper_2505_23963_amd import Batch
    ps = configs.config3_cavities(steps=50000, nfreq=128)
    sig = np.array([p.materials[1].sigma for p in ps])
    picks = [int(np.argmin(sig)), int(np.argsort(sig)[21]), int(np.argsort(sig)[42]), int(np.argmax(sig))]
    print(f"[gpu] 64 cavities f32, 50000 steps; checked: {picks} (sigma {sig[picks]})", flush=True)
    b = Batch(ps)
    orcs = [oracle_lib.Oracle(ps[c]) for c in picks]
    peak = {}
    nthr = max(1, (os.cpu_count() or 4) // len(picks))

    def adv(o, n):
        oracle_lib.set_threads(nthr)
        o.step(n)

    with ThreadPoolExecutor(len(picks)) as ex:
        for done in range(10000, 50001, 10000):
            b.step(10000)
            list(ex.map(lambda o: adv(o, 10000), orcs))
            b.synchronize()
            worst = 0.0
            for c, o in zip(picks, orcs):
                for comp in (2, 4):
                    ref = o.field(comp)[:, 0, 0]
                    peak[(c, comp)] = max(peak.get((c, comp), 0.0), np.linalg.norm(ref))
                    err = np.linalg.norm(b.field(c, comp) - ref) / peak[(c, comp)]
                    worst = max(worst, err)
                    assert err < TOL_F32, (done, c, comp, err)
            print(f"  step {done}: worst field error {worst:.2e}", flush=True)
    for c, o in zip(picks, orcs):
        eg, eo = b.energy(c)[:, 2], o.energy(0)[:, 2]
        ebe = np.max(np.abs(eg - eo)) / np.max(np.abs(eo))
        rel, canc = flux_errors(b.flux(c), o.flux(0), o.flux(0, raw=True)[1])
        print(f"  cavity {c}: bath-energy trace {ebe:.2e}, flux rel-L2 {rel:.2e}, against its scale {canc:.2e}",
              flush=True)
        assert ebe < TOL_F32 and canc < TOL_F32, (c, ebe, canc)


def test_fp32_config2_full_size_200_steps():
    """The whole 256 x 256 x 512 planar cavity in the launch configuration the benchmark times, 200 steps,
    against the FP64 oracle's values on eight sampled columns (tests/golden/make_config2_full_sample.py
    wrote them from the oracle): E, H, P and Y of those columns against the columns' own norms."""
    from paper_2505_23963_amd import Grid
    ref = np.load(os.path.join(HERE, "golden", "config2_full_200.npz"))
    steps, nfreq = int(ref["steps"]), int(ref["nfreq"])
    p = configs.config2_3d(steps=steps, nfreq=nfreq)
    print(f"[gpu] config2 full size f32, {steps} steps", flush=True)
    g = Grid(p)
    g.step(steps)
    g.synchronize()
    xs, ys = ref["columns"][:, 0], ref["columns"][:, 1]
    got = np.stack([g.field(c)[xs, ys, :] for c in range(6)])
    want = ref["fields"]
    for name, sl in (("E", slice(0, 3)), ("H", slice(3, 6))):
        err = np.linalg.norm(got[sl] - want[sl]) / np.linalg.norm(want[sl])
        print(f"  {name} on the sampled columns: {err:.3e}", flush=True)
        assert err < TOL_F32, (name, err)
    nz = p.materials[1].box[1][2] - p.materials[1].box[0][2]
    pol = np.stack([g.polarization(1, c, 0).reshape(256, 256, nz)[xs, ys, :] for c in range(3)])
    bath = np.stack([g.bath(1, c, 0).reshape(p.materials[1].n_bath, 256, 256, nz)[:, xs, ys, :] for c in range(3)])
    for name, a, b in (("P", pol, ref["polarization"]), ("Y", bath, ref["bath"])):
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        print(f"  {name} on the sampled columns: {err:.3e}", flush=True)
        assert err < TOL_F32, (name, err)
    full = np.array([np.linalg.norm(g.field(c)) for c in range(6)])
    assert np.max(np.abs(full - ref["field_norms"]) / ref["field_norms"].max()) < TOL_F32


def test_fp32_config5_full_size_mirror_symmetry():
    """The large 3D layout at its full 512^3 size, in the launch configuration the benchmark times, checked by
    a property that holds at any size: the set-up (periodic x and y, a plane E_x current with a Gaussian
    profile centred between rows ny/2 - 1 and ny/2, materials uniform in x and y) is symmetric under the mirror
    y -> (ny - 1) - y, so after 360 steps (the pulse inside the Lorentz-Bath slab) E_x, E_z, H_y and P_x, P_z
    are even and E_y, H_x, H_z, P_y and the bath of E_y odd under it (a component staggered by half a cell
    along y maps row j to ny - 2 - j).  The updates are mirror images of each other operation by operation,
    so the fields match to rounding (bar 1e-6 of each field's largest value).  Indexing faults that show only
    at full size (block order, 32-bit offsets, region cuts of the 512^2 planes) break the symmetry."""
    import torch
    from paper_2505_23963_amd import Grid
    p = configs.config5_3d_large(steps=360, nfreq=8)
    n = p.n[1]
    print(f"[gpu] config5 full size {p.n} f32, 360 steps, mirror symmetry", flush=True)
    g = Grid(p)
    g.step(360)
    g.synchronize()
    rows = {False: torch.arange(n - 1, -1, -1), True: (n - 2 - torch.arange(n)) % n}
    # component: (sign under the mirror, staggered along y)
    parity = {0: (1, False), 1: (-1, True), 2: (1, False), 3: (-1, True), 4: (1, False), 5: (-1, True)}
    t = torch.empty(p.cells, dtype=torch.float64, device="cuda")
    for c, (sgn, half) in parity.items():
        g.field_into(c, t.data_ptr())
        torch.cuda.synchronize()
        f = t.view(p.n)
        err = (f - sgn * f[:, rows[half].cuda(), :]).abs().max().item()
        scale = f.abs().max().item()
        print(f"  field {c}: max {scale:.3e}, mirror mismatch {err:.3e}", flush=True)
        assert scale > 0 and err <= 1e-6 * scale, (c, err, scale)
    del t
    nz = p.materials[0].box[1][2] - p.materials[0].box[0][2]
    for c, sgn in ((0, 1), (1, -1), (2, 1)):         # P and the bath sit where their E component does
        P = g.polarization(0, c, 0).reshape(n, n, nz)
        err = np.max(np.abs(P - sgn * P[:, rows[c == 1].numpy(), :]))
        print(f"  P{c}: max {np.abs(P).max():.3e}, mirror mismatch {err:.3e}", flush=True)
        assert np.abs(P).max() > 0 and err <= 1e-6 * np.abs(P).max(), (c, err)
    Y = g.bath(0, 1, 0).reshape(-1, n, n, nz)
    err = np.max(np.abs(Y + Y[:, :, rows[True].numpy(), :]))
    print(f"  bath of E_y: max {np.abs(Y).max():.3e}, mirror mismatch {err:.3e}", flush=True)
    assert np.abs(Y).max() > 0 and err <= 1e-6 * np.abs(Y).max()


def test_fp32_config5_full_size_20_steps_sampled_columns(oracle_lib):
    """The 512^3 layout at full size for 20 steps against the oracle on sampled columns.  After 20 steps a
    cell depends only on cells within 2 x 20 of it along x and y, so the oracle runs an 85 x 85 x 512 window
    around each sampled column with the full grid's source profile cut out of the same window (wrapped, x
    and y are periodic) and its centre column must equal the full grid's: E and H over all z, each component
    against the norm of its vector field on the column (the measure of tests/parity_util.py: components fed
    only by diffraction, H_z here at 4e-4 of H_y, carry the FP32 rounding of the dominant one), <= 1e-5.
    Columns at the profile's centre, at its edge and across both wraps."""
    from paper_2505_23963_amd import Grid
    steps, R = 20, 42
    full = configs.config5_3d_large(steps=steps, nfreq=4)
    n = full.n[0]
    prof = full.sources[0].profile.reshape(n, n)
    print(f"[gpu] config5 full size {full.n} f32, {steps} steps, sampled columns", flush=True)
    g = Grid(full)
    g.step(steps)
    g.synchronize()
    fields = {c: g.field(c) for c in range(6)}
    for x0, y0 in ((256, 256), (255, 300), (0, 0), (511, 5)):
        p = configs.config5_3d_large(nx=2 * R + 1, ny=2 * R + 1, steps=steps, nfreq=4)
        ix = (x0 - R + np.arange(2 * R + 1)) % n
        iy = (y0 - R + np.arange(2 * R + 1)) % n
        p.sources[0].profile = np.ascontiguousarray(prof[ix][:, iy]).reshape(2 * R + 1, 2 * R + 1, 1)
        o = oracle_lib.Oracle(p)
        o.step(steps)
        worst = {}
        for name, comps in (("E", (0, 1, 2)), ("H", (3, 4, 5))):
            want = np.stack([o.field(c)[R, R, :] for c in comps])
            got = np.stack([fields[c][x0, y0, :] for c in comps])
            scale = np.linalg.norm(want)
            assert scale > 0
            worst[name] = max(np.linalg.norm(got[i] - want[i]) / scale for i in range(3))
            assert np.linalg.norm(got - want) / scale <= 1e-5 and worst[name] <= 1e-5, (x0, y0, name, worst[name])
        print(f"  column ({x0}, {y0}): worst component E {worst['E']:.2e}, H {worst['H']:.2e}", flush=True)


def test_fp32_config4_full_size_100_steps_sampled_blocks(oracle_lib):
    """The 2D workload at its full 2048^2 size (CPML on every side, the N_b = 64 patch) for 100 steps against
    the oracle on sampled 21 x 21 blocks.  After 100 steps a cell depends on nothing farther than 200 cells,
    so the oracle runs a window of the grid that keeps the full grid's own boundary (its CPML and the source
    line's end) on the sides the block is near and puts its other sides, with their own CPML, more than 200
    cells away.  Blocks by the source line, at its lower end in the corner, and at its upper end.  E_z and
    (H_x, H_y) against their vector fields' norm on the block (reading R11), <= 1e-5."""
    from fdtdb_inputs.problem import PML, PERIODIC, Problem, box
    from paper_2505_23963_amd import Grid
    steps, reach, half = 100, 240, 10
    full = configs.config4_2d(steps=steps, nfreq=4)
    n = full.n[0]
    src = full.sources[0]
    print(f"[gpu] config4 full size {full.n} f32, {steps} steps, sampled blocks", flush=True)
    g = Grid(full)
    g.step(steps)
    g.synchronize()
    fields = {c: g.field(c)[:, :, 0] for c in (2, 3, 4)}
    for x0, y0 in ((60, 1024), (40, 40), (100, 2010)):
        xlo, xhi = 0, x0 + reach                                  # the left boundary is the grid's own
        ylo = 0 if y0 - reach < 0 else y0 - reach
        yhi = n if y0 + reach > n else y0 + reach
        assert xhi <= full.materials[0].box[0][0]                 # the window holds no bath cells
        w = Problem(name="window", ndim=2, n=(xhi - xlo, yhi - ylo, 1), bc=(PML, PML, PERIODIC),
                    pml_cells=(32, 32, 0), dtype="f64", steps=steps)
        # the source line clipped to the window (its ends are the grid's own where the window reaches them)
        s_lo = max(src.box[0][1], ylo) - ylo
        s_hi = min(src.box[1][1], yhi) - ylo
        w.sources.append(configs.gaussian_pulse(2, box((src.box[0][0], src.box[1][0]), (s_lo, s_hi)),
                                                omega_c=src.omega_c, width=src.width))
        o = oracle_lib.Oracle(w)
        o.step(steps)
        bx = slice(x0 - half - xlo, x0 + half + 1 - xlo)
        by = slice(y0 - half - ylo, y0 + half + 1 - ylo)
        gx, gy = slice(x0 - half, x0 + half + 1), slice(y0 - half, y0 + half + 1)
        res = {}
        for name, comps in (("E", (2,)), ("H", (3, 4))):
            want = np.stack([o.field(c)[bx, by, 0] for c in comps])
            got = np.stack([fields[c][gx, gy] for c in comps])
            scale = np.linalg.norm(want)
            assert scale > 0, (x0, y0, name)
            res[name] = np.linalg.norm(got - want) / scale
            assert res[name] <= 1e-5, (x0, y0, name, res[name])
        print(f"  block at ({x0}, {y0}): E {res['E']:.2e}, H {res['H']:.2e}", flush=True)
