"""Boundary checks that need no GPU: the library loads, exports every declared
entry point, and its host-only Table-1 map agrees with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdtdb.h")
LIB = os.path.join(ROOT, "paper_2505_23963_amd", "libfdtdb.so")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fdtdb_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libfdtdb():
    if not os.path.exists(LIB):
        pytest.fail("libfdtdb.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_core_api():
    syms = declared_symbols()
    for s in ["fdtdb_create_grid", "fdtdb_set_lorentz_bath", "fdtdb_add_source", "fdtdb_step", "fdtdb_dft_flux"]:
        assert s in syms


def test_library_exports_every_declared_symbol(libfdtdb):
    missing = [s for s in declared_symbols() if not hasattr(libfdtdb, s)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_2505_23963_amd.fdtdb import SIGNATURES
    bound = {n for n, _, _ in SIGNATURES}
    assert set(declared_symbols()) <= bound


@pytest.mark.parametrize("form", ["uniform", "lorentzian", "gaussian"])
def test_bath_params_matches_oracle_table1(form):
    """Host-only entry point: the library's Table 1 map vs the oracle's."""
    from oracle.closed_form import table1_bath
    from paper_2505_23963_amd import bath_params
    args = (1.0, 0.001, 64, 0.4, 0.4 / 63 / 2, 0.02)
    w, g, k = bath_params(form, *args)
    w2, g2, k2 = table1_bath(form, *args)
    assert np.allclose(w, w2, rtol=0, atol=1e-15)
    assert np.array_equal(g, g2)
    assert np.allclose(k, k2, rtol=1e-14, atol=0)


def test_bath_params_rejects_bad_input():
    from paper_2505_23963_amd import FdtdbError, bath_params
    with pytest.raises(FdtdbError):
        bath_params("uniform", 1.0, 0.0, 1, 0.4, 0.0, 0.02)


def test_version_string(libfdtdb):
    libfdtdb.fdtdb_version.restype = ctypes.c_char_p
    assert b"gfx950" in libfdtdb.fdtdb_version()


def test_product_never_imports_oracle():
    """The product path (package + inputs) must not reach the oracle."""
    for d in ["paper_2505_23963_amd", "fdtdb_inputs"]:
        for dirpath, _, files in os.walk(os.path.join(ROOT, d)):
            for f in files:
                if f.endswith((".py", ".hip", ".h", ".cpp")):
                    txt = open(os.path.join(dirpath, f)).read()
                    assert "import oracle" not in txt and "from oracle" not in txt, f
                    assert "fdtd_oracle" not in txt, f


def _desc(ndim=3, n=(8, 8, 8), courant=0.5, dtype=0):
    from paper_2505_23963_amd.fdtdb import GridDesc
    d = GridDesc()
    d.ndim = ndim
    for a in range(3):
        d.n[a] = n[a]
        d.bc[a] = 1
        d.pml_cells[a] = 0
    d.courant = courant
    d.dtype = dtype
    d.pml_R0 = 1e-8
    return d


@pytest.mark.parametrize("kw, code", [
    (dict(ndim=0), -1), (dict(ndim=4), -1),                         # dimensionality
    (dict(courant=0.0), -1), (dict(courant=0.6), -4),                # 3D vacuum limit 1/sqrt(3)
    (dict(n=(0, 8, 8)), -1),                                         # empty axis
    (dict(n=(2048, 2048, 1024)), -1),                                # beyond 32-bit cell indexing
    (dict(dtype=7), -1),
])
def test_create_grid_rejects_bad_descriptors_before_touching_the_device(libfdtdb, kw, code):
    """Argument checks run on the host before any HIP call, so they are exercised without a GPU."""
    from paper_2505_23963_amd import lib
    L = lib()
    h = ctypes.c_void_p()
    assert L.fdtdb_create_grid(ctypes.byref(_desc(**kw)), ctypes.byref(h)) == code
    assert not h.value
    assert L.fdtdb_last_error()


def test_trainer_and_batch_reject_bad_descriptors(libfdtdb):
    from paper_2505_23963_amd import lib
    from paper_2505_23963_amd.fdtdb import TrainerDesc
    L = lib()
    w = np.array([1.0]); g = np.array([0.01]); k = np.array([0.1])
    P = ctypes.POINTER(ctypes.c_double)

    def desc(**kw):
        d = TrainerDesc()
        d.ntraj, d.nsteps, d.window, d.activation, d.dt, d.n_bath = 4, 128, 64, 0, 0.5, 1
        d.omega_j, d.gamma_j, d.k_j = (a.ctypes.data_as(P) for a in (w, g, k))
        for key, v in kw.items():
            setattr(d, key, v)
        return d

    h = ctypes.c_void_p()
    for bad in (dict(nsteps=100), dict(window=0), dict(window=5000, nsteps=5000), dict(activation=2), dict(dt=0.0),
                dict(n_bath=0), dict(ntraj=0)):
        assert L.fdtdb_trainer_create(ctypes.byref(desc(**bad)), ctypes.byref(h)) == -1, bad
        assert not h.value
    lens = (ctypes.c_int64 * 2)(100, 0)
    assert L.fdtdb_batch_create(2, lens, 0, 0.5, 8, 1e-8, None, ctypes.byref(h)) == -1     # empty cavity
    assert L.fdtdb_batch_create(0, lens, 0, 0.5, 8, 1e-8, None, ctypes.byref(h)) == -1     # no cavities


def test_checkpoint_entry_points_reject_null_arguments(libfdtdb):
    """save_state / load_state check their arguments on the host before any device work."""
    from paper_2505_23963_amd import lib
    L = lib()
    for fn in (L.fdtdb_save_state, L.fdtdb_load_state):
        assert fn(None, b"/tmp/x.state") == -1
        assert b"null" in L.fdtdb_last_error()


def test_allocator_hook_host_checks(libfdtdb):
    """fdtdb_set_allocator needs both callbacks or neither; it touches no device."""
    from paper_2505_23963_amd import lib
    L = lib()
    fa = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)(lambda n, c: None)
    assert L.fdtdb_set_allocator(ctypes.cast(fa, ctypes.c_void_p), None, None) == -1
    assert b"both" in L.fdtdb_last_error()
    assert L.fdtdb_set_allocator(None, None, None) == 0
