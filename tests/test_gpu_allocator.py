"""The device-memory hook (fdtdb_set_allocator) with PyTorch's caching allocator behind it: grids,
batches and trainers take every buffer from it and give every buffer back on destroy, and the
results equal those of the default hipMalloc path bitwise."""
import numpy as np
import pytest

from fdtdb_inputs import configs

pytestmark = pytest.mark.gpu


class Counting:
    def __init__(self, alloc, free):
        self.alloc_, self.free_, self.live, self.calls = alloc, free, set(), 0

    def alloc(self, n):
        p = self.alloc_(n)
        self.live.add(p)
        self.calls += 1
        return p

    def free(self, p):
        self.live.remove(p)
        self.free_(p)


def _run_objects():
    from paper_2505_23963_amd import Batch, Grid, Trainer
    p = configs.config2_3d(nx=8, ny=8, steps=0, nfreq=16, dtype="f32")
    g = Grid(p, graph_chunk=8)
    g.step(40)
    out = {f"grid{c}": g.field(c) for c in range(6)}
    out["flux"] = g.flux(0)
    g.close()
    ps = configs.config3_cavities(ncav=2, steps=64, dtype="f32", nfreq=16, lengths=[1500, 1700])
    b = Batch(ps, tiling=(16, 256))
    b.step(64)
    out["batch"] = b.field(0, 2)
    b.close()
    rng = np.random.default_rng(0)
    E = rng.standard_normal((128, 8)).astype(np.float32) * 1e-2
    P = np.cumsum(E, axis=0).astype(np.float32) * 1e-3
    t = Trainer(8, 128, 64, 0.5, np.array([1.0]), np.array([0.01]), np.array([0.05]), activation="identity")
    t.load(E, P)
    out["targets"] = t.targets()
    del t
    return out


def test_torch_caching_allocator_backs_every_object():
    import gc
    import torch
    from paper_2505_23963_amd import set_allocator, torch_allocator
    print("[gpu] allocator: default path", flush=True)
    want = _run_objects()
    gc.collect()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(0)
    cnt = Counting(*torch_allocator(0))
    set_allocator(cnt.alloc, cnt.free)
    try:
        print("[gpu] allocator: torch caching allocator", flush=True)
        got = _run_objects()
        gc.collect()
    finally:
        set_allocator()
    assert cnt.calls > 0
    assert not cnt.live, f"{len(cnt.live)} blocks not given back"
    assert torch.cuda.memory_allocated(0) == base
    for k, v in want.items():
        assert np.array_equal(got[k], v), k
