"""ctypes binding of libfdtdb (the C-ABI declared in include/fdtdb.h).

Argument marshalling only: every step of the time-stepping path runs in the
library's HIP kernels.  The binding refuses to run without the built
library; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtdb.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_UNSTABLE, E_DIVERGED, E_STATE = 0, -1, -2, -3, -4, -5, -6
F32, F64 = 0, 1
BC_PML, BC_PERIODIC, BC_CLOSED = 0, 1, 2
_FORMS = {"uniform": 0, "lorentzian": 1, "gaussian": 2}


class FdtdbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fdtdb status {status}: {msg}")
        self.status = status


class Box(C.Structure):
    _fields_ = [("lo", C.c_int64 * 3), ("hi", C.c_int64 * 3)]


class GridDesc(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int64 * 3), ("courant", C.c_double), ("dtype", C.c_int),
                ("bc", C.c_int * 3), ("pml_cells", C.c_int * 3), ("pml_R0", C.c_double),
                ("hip_stream", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("cells", C.c_int64), ("dispersive_cells", C.c_int64), ("bath_cells", C.c_int64),
                ("bytes_per_step", C.c_double), ("bytes_per_step_e", C.c_double), ("bytes_per_step_h", C.c_double),
                ("launches_per_step", C.c_int)]


class KernelRecord(C.Structure):
    _fields_ = [("region", C.c_int), ("phase", C.c_int), ("kind", C.c_int), ("n_bath", C.c_int), ("pml", C.c_int),
                ("cells", C.c_int64), ("bytes", C.c_double), ("ms_total", C.c_double), ("launches", C.c_int64)]


_lib = None
_dp = C.POINTER(C.c_double)

# (name, restype, argtypes) of every entry point of include/fdtdb.h
SIGNATURES = [
    ("fdtdb_create_grid", C.c_int, [C.POINTER(GridDesc), C.POINTER(C.c_void_p)]),
    ("fdtdb_destroy_grid", C.c_int, [C.c_void_p]),
    ("fdtdb_set_eps_inf", C.c_int, [C.c_void_p, C.POINTER(Box), C.c_double, C.POINTER(C.c_int)]),
    ("fdtdb_set_drude", C.c_int, [C.c_void_p, C.POINTER(Box), C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int)]),
    ("fdtdb_set_lorentz_bath", C.c_int, [C.c_void_p, C.POINTER(Box), C.c_double, C.c_double, C.c_double, _dp,
                                         C.c_double, C.c_int, _dp, _dp, _dp, C.POINTER(C.c_int)]),
    ("fdtdb_set_multi_term", C.c_int, [C.c_void_p, C.POINTER(Box), C.c_double, C.c_int, C.POINTER(C.c_int), _dp, _dp,
                                       _dp, C.POINTER(C.c_int)]),
    ("fdtdb_get_polarization_term", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, _dp]),
    ("fdtdb_bath_params", C.c_int, [C.c_int, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double, C.c_double,
                                    _dp, _dp, _dp]),
    ("fdtdb_set_bath_closure", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_float), C.c_int, _dp]),
    ("fdtdb_set_bath_storage", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_double]),
    ("fdtdb_set_bath_thermal", C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_uint64]),
    ("fdtdb_set_bath_anharmonic", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int]),
    ("fdtdb_get_closure_state", C.c_int, [C.c_void_p, C.c_int, C.c_int, _dp]),
    ("fdtdb_add_source", C.c_int, [C.c_void_p, C.c_int, C.POINTER(Box), C.c_double, C.c_double, C.c_double, _dp,
                                   C.POINTER(C.c_int)]),
    ("fdtdb_add_dft_flux", C.c_int, [C.c_void_p, C.c_int, C.POINTER(Box), C.c_int, _dp, C.POINTER(C.c_int)]),
    ("fdtdb_add_energy_monitor", C.c_int, [C.c_void_p, C.POINTER(Box), C.c_int, C.POINTER(C.c_int)]),
    ("fdtdb_step", C.c_int, [C.c_void_p, C.c_int64]),
    ("fdtdb_pair_bloch", C.c_int, [C.c_void_p, C.c_void_p, _dp]),
    ("fdtdb_synchronize", C.c_int, [C.c_void_p]),
    ("fdtdb_steps_done", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("fdtdb_set_graph", C.c_int, [C.c_void_p, C.c_int]),
    ("fdtdb_set_allocator", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("fdtdb_save_state", C.c_int, [C.c_void_p, C.c_char_p]),
    ("fdtdb_load_state", C.c_int, [C.c_void_p, C.c_char_p]),
    ("fdtdb_dft_flux", C.c_int, [C.c_void_p, C.c_int, _dp, _dp]),
    ("fdtdb_energy", C.c_int, [C.c_void_p, C.c_int, _dp, C.c_int64, C.POINTER(C.c_int64)]),
    ("fdtdb_get_field", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int]),
    ("fdtdb_set_field", C.c_int, [C.c_void_p, C.c_int, _dp]),
    ("fdtdb_get_polarization", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, _dp]),
    ("fdtdb_get_bath", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, _dp]),
    ("fdtdb_get_stats", C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    ("fdtdb_set_profiling", C.c_int, [C.c_void_p, C.c_int]),
    ("fdtdb_kernel_records", C.c_int, [C.c_void_p, C.POINTER(KernelRecord), C.c_int, C.POINTER(C.c_int)]),
    ("fdtdb_batch_create", C.c_int, [C.c_int, C.POINTER(C.c_int64), C.c_int, C.c_double, C.c_int, C.c_double,
                                     C.c_void_p, C.POINTER(C.c_void_p)]),
    ("fdtdb_batch_destroy", C.c_int, [C.c_void_p]),
    ("fdtdb_batch_set_drude", C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double]),
    ("fdtdb_batch_set_lorentz_bath", C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_double, C.c_double,
                                               C.c_double, C.c_double, C.c_int, _dp, _dp, _dp]),
    ("fdtdb_batch_add_source", C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_double, C.c_double]),
    ("fdtdb_batch_add_dft_flux", C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, _dp]),
    ("fdtdb_batch_add_energy_monitor", C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_int]),
    ("fdtdb_batch_set_tiling", C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    ("fdtdb_batch_get_tiling", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("fdtdb_batch_step", C.c_int, [C.c_void_p, C.c_int64]),
    ("fdtdb_batch_synchronize", C.c_int, [C.c_void_p]),
    ("fdtdb_batch_steps_done", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("fdtdb_batch_get_field", C.c_int, [C.c_void_p, C.c_int, C.c_int, _dp]),
    ("fdtdb_batch_dft_flux", C.c_int, [C.c_void_p, C.c_int, _dp]),
    ("fdtdb_batch_energy", C.c_int, [C.c_void_p, C.c_int, _dp, C.c_int64, C.POINTER(C.c_int64)]),
    ("fdtdb_batch_energy_noalloc", C.c_int, [C.c_void_p, C.c_int, _dp, C.c_int64, C.POINTER(C.c_int64)]),
    ("fdtdb_batch_last_error", C.c_char_p, []),
    ("fdtdb_add_probe", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int64), C.c_int64,
                                  C.POINTER(C.c_int)]),
    ("fdtdb_probe_data", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    ("fdtdb_trainer_create", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    ("fdtdb_trainer_destroy", C.c_int, [C.c_void_p]),
    ("fdtdb_trainer_load", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    ("fdtdb_trainer_get_scales", C.c_int, [C.c_void_p, _dp]),
    ("fdtdb_trainer_get_targets", C.c_int, [C.c_void_p, _dp]),
    ("fdtdb_trainer_set_weights", C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    ("fdtdb_trainer_get_weights", C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    ("fdtdb_trainer_set_activation", C.c_int, [C.c_void_p, C.c_int, C.c_double]),
    ("fdtdb_trainer_loss_grad", C.c_int, [C.c_void_p, _dp, _dp]),
    ("fdtdb_trainer_train", C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_double, _dp]),
    ("fdtdb_trainer_last_error", C.c_char_p, []),
    ("fdtdb_last_error", C.c_char_p, []),
    ("fdtdb_version", C.c_char_p, []),
]


def lib():
    """Load libfdtdb.so; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_2505_23963_amd.build)")
        # PyTorch ships its own HIP runtime under the same soname as the system one this library links;
        # the first loaded serves the whole process, and PyTorch cannot start its GPU support on a runtime
        # loaded before it.  Loading PyTorch first keeps one runtime that both use (streams and the
        # caching allocator are shared with it).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_allocator_refs = []   # callback objects of every allocator ever set (objects may outlive a reset)


def set_allocator(alloc=None, free=None):
    """Device memory source of grids, batches and trainers created from now on (fdtdb_set_allocator):
    alloc(nbytes) -> device address (int, 0 on failure), free(address).  No arguments: hipMalloc."""
    if alloc is None and free is None:
        _check(lib().fdtdb_set_allocator(None, None, None))
        return
    fa = _ALLOC_FN(lambda n, ctx: alloc(n) or None)
    ff = _FREE_FN(lambda p, ctx: free(p))
    _allocator_refs.append((fa, ff))
    _check(lib().fdtdb_set_allocator(C.cast(fa, C.c_void_p), C.cast(ff, C.c_void_p), None))


def torch_allocator(device: int = 0):
    """alloc / free callables backed by PyTorch's caching allocator on one device."""
    import torch

    def alloc(n):
        return torch.cuda.caching_allocator_alloc(int(n), device)

    def free(p):
        torch.cuda.caching_allocator_delete(p)

    return alloc, free


def _check(st: int):
    if st != OK:
        raise FdtdbError(st, lib().fdtdb_last_error().decode())


def _box(b) -> Box:
    x = Box()
    for a in range(3):
        x.lo[a] = int(b[0][a])
        x.hi[a] = int(b[1][a])
    return x


def _arr(a) -> Optional[np.ndarray]:
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=np.float64).ravel()


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_dp)


CLOSURE_WIDTH = 32
_CLOSURE_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def closure_weights(params: dict) -> np.ndarray:
    """Flat FP32 closure weights in the library layout W1[32][7], b1, W2[32][32], b2, W3[5][32], b3."""
    w = np.concatenate([np.asarray(params[k], np.float32).ravel() for k in _CLOSURE_ORDER])
    if w.size != 32 * 7 + 32 + 32 * 32 + 32 + 5 * 32 + 5:
        raise ValueError("closure weights must have width 32")
    return w


def bath_params(form: str, omega0: float, gamma0: float, n_bath: int, width: float, bath_gamma: float,
                dephasing: float):
    """Table 1 map computed by the library."""
    w, g, k = (np.zeros(n_bath) for _ in range(3))
    _check(lib().fdtdb_bath_params(_FORMS[form], omega0, gamma0, n_bath, width, bath_gamma, dephasing,
                                   _ptr(w), _ptr(g), _ptr(k)))
    return w, g, k


class Grid:
    """A device grid built from an fdtdb_inputs Problem description.  A problem with Bloch phases
    (problem.bloch) becomes two device grids coupled by fdtdb_pair_bloch, the real (h) and imaginary
    (h_im) parts of complex fields: fields, material state and the flux's raw transforms then read
    back complex, energies as the sum over both parts."""

    def __init__(self, problem, stream: Optional[int] = None, graph_chunk: int = 0, dtype: Optional[str] = None,
                 closures: Optional[dict] = None):
        """closures: {material index: {"weights": 1477 floats, "scales": (s_E, s_P, s_V, s_S)}}."""
        self.p = problem
        self._probes = {}
        self.h_im = None
        self.h, self.mat_ids = self._build(problem, stream, dtype, closures, 0)
        if problem.bloch is not None:
            if closures:
                raise ValueError("learned closures are not available on Bloch grids")
            self.h_im, _ = self._build(problem, stream, dtype, None, 1)
            ph = _arr(problem.bloch)
            _check(lib().fdtdb_pair_bloch(self.h, self.h_im, _ptr(ph)))
        elif graph_chunk:
            _check(lib().fdtdb_set_graph(self.h, int(graph_chunk)))

    @property
    def _parts(self):
        return [self.h] if self.h_im is None else [self.h, self.h_im]

    def _both(self, fn):
        """fn(handle) of the real part, + 1j fn(handle) of the imaginary part of a Bloch grid"""
        v = fn(self.h)
        return v if self.h_im is None else v + 1j * fn(self.h_im)

    @staticmethod
    def _build(problem, stream, dtype, closures, part):
        """One device grid with the problem's set-up; part 1 (imaginary part of a Bloch grid) takes the
        imaginary parts of the source profiles (sources without one drive the real part only)."""
        L = lib()
        d = GridDesc()
        d.ndim = problem.ndim
        for a in range(3):
            d.n[a] = int(problem.n[a])
            d.bc[a] = int(problem.bc[a])
            d.pml_cells[a] = int(problem.pml_cells[a])
        d.courant = problem.courant
        dt = dtype or problem.dtype
        d.dtype = F64 if dt == "f64" else F32
        d.pml_R0 = problem.pml_R0
        d.hip_stream = stream
        h = C.c_void_p()
        _check(L.fdtdb_create_grid(C.byref(d), C.byref(h)))
        mat_ids = []
        for m in problem.materials:
            kind = type(m).__name__
            mid = C.c_int(-1)
            b = _box(m.box)
            if kind == "Dielectric":
                _check(L.fdtdb_set_eps_inf(h, C.byref(b), m.eps_inf, C.byref(mid)))
            elif kind == "Drude":
                _check(L.fdtdb_set_drude(h, C.byref(b), m.omega_p, m.gamma, m.eps_inf, C.byref(mid)))
            elif kind == "LorentzBath":
                if m.n_bath and m.form is not None:
                    wj, gj, kj = bath_params(m.form, m.omega0, m.gamma0, m.n_bath, m.width, m.bath_gamma,
                                             m.dephasing)
                else:
                    wj, gj, kj = _arr(m.omega_j), _arr(m.gamma_j), _arr(m.k_j)
                sig = _arr(m.sigma_cells)
                _check(L.fdtdb_set_lorentz_bath(h, C.byref(b), m.omega0, m.gamma0, m.eps_inf, _ptr(sig),
                                                m.sigma, m.n_bath, _ptr(wj), _ptr(gj), _ptr(kj), C.byref(mid)))
                if m.bath_storage is not None:
                    _check(L.fdtdb_set_bath_storage(h, mid.value, {"f16": 1, "bf16": 2}[m.bath_storage],
                                                    float(m.bath_scale)))
                if getattr(m, "kT", 0.0):
                    _check(L.fdtdb_set_bath_thermal(h, mid.value, float(m.kT), int(m.noise_seed)))
                if getattr(m, "anharmonic", None) is not None:
                    lam = np.ascontiguousarray(m.anharmonic, np.float64)
                    _check(L.fdtdb_set_bath_anharmonic(h, mid.value, _ptr(lam), len(lam)))
            elif kind == "MultiPole":
                nt = len(m.kinds)
                kinds = (C.c_int * nt)(*[{"lorentz": 0, "drude": 1}[k] for k in m.kinds])
                om, ga, sg = (np.ascontiguousarray(v, np.float64) for v in (m.omega, m.gamma, m.sigma))
                _check(L.fdtdb_set_multi_term(h, C.byref(b), m.eps_inf, nt, kinds, _ptr(om), _ptr(ga), _ptr(sg),
                                              C.byref(mid)))
            else:
                raise TypeError(kind)
            mat_ids.append(mid.value)
        for mi, cl in (closures or {}).items():
            w = np.ascontiguousarray(cl["weights"], dtype=np.float32).ravel()
            sc = _arr(cl["scales"])
            _check(L.fdtdb_set_bath_closure(h, mat_ids[mi], w.ctypes.data_as(C.POINTER(C.c_float)), 32,
                                            _ptr(sc)))
        for s in problem.sources:
            pr = s.profile if part == 0 else s.profile_im
            if part == 1 and pr is None:
                continue
            prof = _arr(pr)
            _check(L.fdtdb_add_source(h, s.comp, C.byref(_box(s.box)), s.omega_c, s.width, s.amplitude,
                                      _ptr(prof), None))
        for dm in problem.dfts:
            om = _arr(dm.omega)
            _check(L.fdtdb_add_dft_flux(h, dm.axis, C.byref(_box(dm.box)), len(om), _ptr(om), None))
        for e in problem.energies:
            _check(L.fdtdb_add_energy_monitor(h, C.byref(_box(e.box)), e.every, None))
        return h, mat_ids

    def close(self):
        for name in ("h_im", "h"):
            if getattr(self, name, None):
                lib().fdtdb_destroy_grid(getattr(self, name))
                setattr(self, name, None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int):
        _check(lib().fdtdb_step(self.h, int(n)))

    def synchronize(self):
        for h in self._parts:
            _check(lib().fdtdb_synchronize(h))

    @property
    def steps_done(self) -> int:
        s = C.c_int64()
        _check(lib().fdtdb_steps_done(self.h, C.byref(s)))
        return s.value

    def field(self, comp: int) -> np.ndarray:
        def one(h):
            out = np.zeros(self.p.cells, np.float64)
            _check(lib().fdtdb_get_field(h, comp, out.ctypes.data_as(C.c_void_p), 0))
            return out.reshape(self.p.n)
        return self._both(one)

    def field_into(self, comp: int, device_ptr: int, part: int = 0):
        """Write a field component (FP64, C order) into device memory at device_ptr (e.g. a torch
        float64 CUDA tensor's data_ptr() of n[0]*n[1]*n[2] elements); part 1: the imaginary part of a
        Bloch grid."""
        _check(lib().fdtdb_get_field(self._parts[part], comp, C.c_void_p(device_ptr), 1))

    def set_field(self, comp: int, values):
        _check(lib().fdtdb_set_field(self.h, comp, _ptr(_arr(np.real(values)))))
        if self.h_im is not None:
            _check(lib().fdtdb_set_field(self.h_im, comp, _ptr(_arr(np.imag(values)))))

    def _mcells(self, mi):
        b = self.p.materials[mi].box
        return int(np.prod([b[1][a] - b[0][a] for a in range(3)]))

    def polarization(self, mi: int, comp: int, level: int = 0) -> np.ndarray:
        def one(h):
            out = np.zeros(self._mcells(mi), np.float64)
            _check(lib().fdtdb_get_polarization(h, self.mat_ids[mi], comp, level, _ptr(out)))
            return out
        return self._both(one)

    def pole(self, mi: int, comp: int, term: int, level: int = 0) -> np.ndarray:
        """Polarization of one term of a multi-term material."""
        def one(h):
            out = np.zeros(self._mcells(mi), np.float64)
            _check(lib().fdtdb_get_polarization_term(h, self.mat_ids[mi], comp, level, term, _ptr(out)))
            return out
        return self._both(one)

    def bath(self, mi: int, comp: int, level: int = 0) -> np.ndarray:
        nb = self.p.materials[mi].n_bath

        def one(h):
            out = np.zeros(nb * self._mcells(mi), np.float64)
            _check(lib().fdtdb_get_bath(h, self.mat_ids[mi], comp, level, _ptr(out)))
            return out.reshape(nb, -1)
        return self._both(one)

    def add_probe(self, mi: int, comp: int, cells, nsteps: int) -> int:
        """Record E^{n+1/2} and the new P at material-box cells for steps [0, nsteps)."""
        c = np.ascontiguousarray(cells, np.int64)
        pid = C.c_int(-1)
        _check(lib().fdtdb_add_probe(self.h, self.mat_ids[mi], comp, len(c), c.ctypes.data_as(C.POINTER(C.c_int64)),
                                     int(nsteps), C.byref(pid)))
        self._probes[pid.value] = (len(c), int(nsteps))
        return pid.value

    def probe_data(self, pid: int):
        """(E, P) records, [nsteps][ncells] float32 host arrays."""
        n, T = self._probes[pid]
        E = np.zeros((T, n), np.float32)
        P = np.zeros((T, n), np.float32)
        _check(lib().fdtdb_probe_data(self.h, pid, E.ctypes.data, P.ctypes.data, 0))
        return E, P

    def closure_state(self, mi: int, comp: int) -> np.ndarray:
        out = np.zeros(4 * self._mcells(mi), np.float64)
        _check(lib().fdtdb_get_closure_state(self.h, self.mat_ids[mi], comp, _ptr(out)))
        return out.reshape(-1, 4)

    def flux(self, mid: int, raw: bool = False):
        d = self.p.dfts[mid]
        nf = len(d.omega)
        npts = int(np.prod([d.box[1][a] - d.box[0][a] for a in range(3)]))
        out = np.zeros(nf, np.float64)
        r = np.zeros(4 * npts * nf * 2, np.float64) if raw else None
        _check(lib().fdtdb_dft_flux(self.h, mid, _ptr(out), _ptr(r)))
        if raw:
            rr = r.reshape(4, npts, nf, 2)
            tr = rr[..., 0] + 1j * rr[..., 1]
            if self.h_im is not None:    # transforms of the complex fields: real part's + 1j * imaginary part's
                ri = np.zeros(4 * npts * nf * 2, np.float64)
                _check(lib().fdtdb_dft_flux(self.h_im, mid, None, _ptr(ri)))
                ri = ri.reshape(4, npts, nf, 2)
                tr = tr + 1j * (ri[..., 0] + 1j * ri[..., 1])
            return out, tr
        return out

    def energy(self, mid: int) -> np.ndarray:
        """[field, polarization, bath] per sample (the sum over both parts of a Bloch grid)"""
        tot = None
        for h in self._parts:
            n = C.c_int64()
            _check(lib().fdtdb_energy(h, mid, None, 0, C.byref(n)))
            out = np.zeros(3 * max(n.value, 1), np.float64)
            _check(lib().fdtdb_energy(h, mid, _ptr(out), n.value, C.byref(n)))
            e = out[:3 * n.value].reshape(-1, 3)
            tot = e if tot is None else tot + e
        return tot

    def save_state(self, path: str):
        """Write the whole time-stepping state to a file (fdtdb_save_state)."""
        _check(lib().fdtdb_save_state(self.h, os.fsencode(path)))

    def load_state(self, path: str):
        """Resume from a file written by save_state on a grid of the same set-up."""
        _check(lib().fdtdb_load_state(self.h, os.fsencode(path)))

    def set_profiling(self, on, bath_only: bool = False):
        """Events around every E/H launch (on), or only around the E launches of Lorentz-Bath and
        learned-closure materials."""
        _check(lib().fdtdb_set_profiling(self.h, 0 if not on else (2 if bath_only else 1)))

    def kernel_records(self):
        n = C.c_int()
        _check(lib().fdtdb_kernel_records(self.h, None, 0, C.byref(n)))
        arr = (KernelRecord * max(n.value, 1))()
        _check(lib().fdtdb_kernel_records(self.h, arr, n.value, C.byref(n)))
        return [{f: getattr(arr[i], f) for f, _ in KernelRecord._fields_} for i in range(n.value)]

    def stats(self) -> dict:
        s = Stats()
        _check(lib().fdtdb_get_stats(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}


def _bcheck(st: int):
    if st != OK:
        raise FdtdbError(st, lib().fdtdb_batch_last_error().decode())


class Batch:
    """Many independent 1D cavities advanced together (fdtdb_batch_* entry points).

    Built from a list of 1D Problem descriptions that share dtype, courant and
    CPML thickness; each may hold one Drude medium (possibly several boxes with
    equal parameters), one Lorentz-Bath box, one source cell, one DFT node and one
    energy box.
    """

    def __init__(self, problems, stream: Optional[int] = None, tiling=None, dtype: Optional[str] = None):
        L = lib()
        self.ps = list(problems)
        p0 = self.ps[0]
        n = len(self.ps)
        lens = (C.c_int64 * n)(*[int(p.n[0]) for p in self.ps])
        dt = dtype or p0.dtype
        h = C.c_void_p()
        pml = int(p0.pml_cells[0]) if p0.bc[0] == BC_PML else 0
        _bcheck(L.fdtdb_batch_create(n, lens, F64 if dt == "f64" else F32, p0.courant, pml, p0.pml_R0, stream,
                                     C.byref(h)))
        self.h = h
        for c, p in enumerate(self.ps):
            for m in p.materials:
                kind = type(m).__name__
                lo, hi = int(m.box[0][0]), int(m.box[1][0])
                if kind == "Drude":
                    _bcheck(L.fdtdb_batch_set_drude(self.h, c, lo, hi, m.omega_p, m.gamma, m.eps_inf))
                elif kind == "LorentzBath":
                    if m.n_bath and m.form is not None:
                        wj, gj, kj = bath_params(m.form, m.omega0, m.gamma0, m.n_bath, m.width, m.bath_gamma,
                                                 m.dephasing)
                    else:
                        wj, gj, kj = _arr(m.omega_j), _arr(m.gamma_j), _arr(m.k_j)
                    if m.sigma_cells is not None:
                        raise ValueError("batched cavities take a uniform sigma")
                    if getattr(m, "kT", 0.0) or getattr(m, "anharmonic", None) is not None or m.bath_storage:
                        raise ValueError("batched cavities take a harmonic bath at zero temperature in the state type")
                    _bcheck(L.fdtdb_batch_set_lorentz_bath(self.h, c, lo, hi, m.omega0, m.gamma0, m.eps_inf, m.sigma,
                                                           m.n_bath, _ptr(wj), _ptr(gj), _ptr(kj)))
                else:
                    raise TypeError(kind)
            for s in p.sources:
                _bcheck(L.fdtdb_batch_add_source(self.h, c, int(s.box[0][0]), s.omega_c, s.width, s.amplitude))
            for d in p.dfts:
                om = _arr(d.omega)
                _bcheck(L.fdtdb_batch_add_dft_flux(self.h, c, int(d.box[0][0]), len(om), _ptr(om)))
            for e in p.energies:
                _bcheck(L.fdtdb_batch_add_energy_monitor(self.h, c, int(e.box[0][0]), int(e.box[1][0]), e.every))
        if tiling is not None:
            _bcheck(L.fdtdb_batch_set_tiling(self.h, int(tiling[0]), int(tiling[1])))

    def close(self):
        if getattr(self, "h", None):
            lib().fdtdb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def tiling(self):
        a, b = C.c_int(), C.c_int()
        _bcheck(lib().fdtdb_batch_get_tiling(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def step(self, n: int):
        _bcheck(lib().fdtdb_batch_step(self.h, int(n)))

    def synchronize(self):
        _bcheck(lib().fdtdb_batch_synchronize(self.h))

    def field(self, cav: int, comp: int) -> np.ndarray:
        out = np.zeros(int(self.ps[cav].n[0]), np.float64)
        _bcheck(lib().fdtdb_batch_get_field(self.h, cav, comp, _ptr(out)))
        return out

    def flux(self, cav: int) -> np.ndarray:
        nf = len(self.ps[cav].dfts[0].omega)
        out = np.zeros(nf, np.float64)
        _bcheck(lib().fdtdb_batch_dft_flux(self.h, cav, _ptr(out)))
        return out

    def energy(self, cav: int) -> np.ndarray:
        n = C.c_int64()
        _bcheck(lib().fdtdb_batch_energy(self.h, cav, None, 0, C.byref(n)))
        out = np.zeros(3 * max(n.value, 1), np.float64)
        _bcheck(lib().fdtdb_batch_energy(self.h, cav, _ptr(out), n.value, C.byref(n)))
        return out[:3 * n.value].reshape(-1, 3)


class TrainerDesc(C.Structure):
    _fields_ = [("ntraj", C.c_int64), ("nsteps", C.c_int64), ("window", C.c_int), ("activation", C.c_int),
                ("dt", C.c_double), ("n_bath", C.c_int), ("omega_j", _dp), ("gamma_j", _dp), ("k_j", _dp),
                ("hip_stream", C.c_void_p)]


def _tcheck(st: int):
    if st != OK:
        raise FdtdbError(st, lib().fdtdb_trainer_last_error().decode())


class Trainer:
    """GPU trainer of the learned closure (fdtdb_trainer_* entry points)."""

    def __init__(self, ntraj: int, nsteps: int, window: int, dt: float, omega_j, gamma_j, k_j,
                 activation: str = "tanh", stream: Optional[int] = None):
        L = lib()
        self._bath = [_arr(omega_j), _arr(gamma_j), _arr(k_j)]
        d = TrainerDesc()
        d.ntraj, d.nsteps, d.window = int(ntraj), int(nsteps), int(window)
        d.activation = {"tanh": 0, "identity": 1}[activation]
        d.dt = float(dt)
        d.n_bath = len(self._bath[0])
        d.omega_j, d.gamma_j, d.k_j = (_ptr(a) for a in self._bath)
        d.hip_stream = stream
        h = C.c_void_p()
        _tcheck(L.fdtdb_trainer_create(C.byref(d), C.byref(h)))
        self.h = h
        self.N, self.T = int(ntraj), int(nsteps)

    def __del__(self):
        if getattr(self, "h", None):
            lib().fdtdb_trainer_destroy(self.h)
            self.h = None

    def load(self, E: np.ndarray, P: np.ndarray):
        """E, P: [nsteps][ntraj] records (float32)."""
        E = np.ascontiguousarray(E, np.float32)
        P = np.ascontiguousarray(P, np.float32)
        if E.shape != (self.T, self.N) or P.shape != (self.T, self.N):
            raise ValueError("records must be [nsteps][ntraj]")
        _tcheck(lib().fdtdb_trainer_load(self.h, E.ctypes.data, P.ctypes.data, 0))

    def load_from_grid(self, grid: "Grid", pid: int):
        E, P = grid.probe_data(pid)
        self.load(E, P)

    def scales(self) -> np.ndarray:
        out = np.zeros(4, np.float64)
        _tcheck(lib().fdtdb_trainer_get_scales(self.h, _ptr(out)))
        return out

    def targets(self) -> np.ndarray:
        out = np.zeros((self.T, self.N), np.float64)
        _tcheck(lib().fdtdb_trainer_get_targets(self.h, _ptr(out)))
        return out

    def set_weights(self, w):
        w = np.ascontiguousarray(w, np.float32).ravel()
        _tcheck(lib().fdtdb_trainer_set_weights(self.h, w.ctypes.data_as(C.POINTER(C.c_float))))

    def weights(self) -> np.ndarray:
        w = np.zeros(32 * 7 + 32 + 32 * 32 + 32 + 5 * 32 + 5, np.float32)
        _tcheck(lib().fdtdb_trainer_get_weights(self.h, w.ctypes.data_as(C.POINTER(C.c_float))))
        return w

    def set_activation(self, activation: str, eps: float = 1e-4):
        """Switch the training activation; identity -> tanh carries the weights over (eps scaling)."""
        _tcheck(lib().fdtdb_trainer_set_activation(self.h, {"tanh": 0, "identity": 1}[activation], float(eps)))

    def loss_grad(self):
        loss = np.zeros(1, np.float64)
        g = np.zeros(32 * 7 + 32 + 32 * 32 + 32 + 5 * 32 + 5, np.float64)
        _tcheck(lib().fdtdb_trainer_loss_grad(self.h, _ptr(loss), _ptr(g)))
        return float(loss[0]), g

    def train(self, epochs: int, lr: float, lr_decay: float = 1.0) -> np.ndarray:
        out = np.zeros(max(int(epochs), 1), np.float64)
        _tcheck(lib().fdtdb_trainer_train(self.h, int(epochs), float(lr), float(lr_decay), _ptr(out)))
        return out[:int(epochs)]
