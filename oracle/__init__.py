"""FDTD-Bath oracle: plain CPU FP64 reference (TEST INFRASTRUCTURE ONLY).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library.  The time step itself
is plain C (fdtd_oracle.c, loops over cells in the paper's order); this
module builds it with gcc, drives it through ctypes, and maps a workload
description onto it.  Closed forms used to pin it live in closed_form.py; the
learned-closure reference (forward, backpropagation through time, Adam) lives
in closure.py.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

from . import closed_form

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdtd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math: IEEE FP64)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-std=c11", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.c_int, C.c_long, C.c_long, C.c_long, C.c_double]
        L.or_set_boundary.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double]
        L.or_add_dielectric.argtypes = [C.c_void_p, _lp, _lp, C.c_double]
        L.or_add_drude.argtypes = [C.c_void_p, _lp, _lp, C.c_double, C.c_double, C.c_double]
        L.or_add_lorentz_bath.argtypes = [C.c_void_p, _lp, _lp, C.c_double, C.c_double, C.c_double,
                                          C.c_void_p, C.c_double, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_add_multipole.argtypes = [C.c_void_p, _lp, _lp, C.c_double, C.c_int,
                                       np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS"), _dp, _dp, _dp]
        L.or_get_P_pole.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, _dp]
        L.or_set_P_pole.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, _dp]
        L.or_add_closure.argtypes = [C.c_void_p, _lp, _lp, C.c_double, C.c_double, C.c_double, C.c_void_p,
                                     C.c_double, C.c_double, C.c_int, _dp, _dp]
        L.or_add_source.argtypes = [C.c_void_p, C.c_int, _lp, _lp, C.c_double, C.c_double, C.c_double, C.c_void_p]
        L.or_add_dft.argtypes = [C.c_void_p, C.c_int, _lp, _lp, C.c_int, _dp]
        L.or_add_energy.argtypes = [C.c_void_p, _lp, _lp, C.c_int]
        L.or_step.argtypes = [C.c_void_p, C.c_long]
        L.or_pair_bloch.argtypes = [C.c_void_p, C.c_void_p, _dp]
        L.or_get_step.restype = C.c_long
        L.or_get_step.argtypes = [C.c_void_p]
        L.or_set_threads.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_field.argtypes = [C.c_void_p, C.c_int, _dp]
        L.or_set_field.argtypes = [C.c_void_p, C.c_int, _dp]
        L.or_get_P.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _dp]
        L.or_get_Y.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _dp]
        L.or_get_hidden.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp]
        L.or_set_P.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _dp]
        L.or_set_Y.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _dp]
        L.or_drive_material.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp, C.c_long, _dp]
        L.or_set_bath_thermal.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_uint64]
        L.or_set_bath_anharmonic.argtypes = [C.c_void_p, C.c_int, _dp]
        _up = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
        L.or_philox.argtypes = [_up, _up, _up]
        L.or_get_dft.argtypes = [C.c_void_p, C.c_int, _dp, C.c_void_p]
        L.or_energy_count.restype = C.c_long
        L.or_energy_count.argtypes = [C.c_void_p, C.c_int]
        L.or_get_energy.argtypes = [C.c_void_p, C.c_int, _dp]
        L.or_destroy.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads for the oracle's cell loops (OpenMP; the default is OMP_NUM_THREADS or all cores).  The
    results do not depend on it.  n < 1 leaves it unchanged; returns the count in force."""
    return int(lib().or_set_threads(int(n)))


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.c_void_p)


def _box(b):
    return np.asarray(b[0], dtype=np.int64), np.asarray(b[1], dtype=np.int64)


def bath_arrays(mat):
    """(omega_j, gamma_j, k_j) of a LorentzBath description, via the oracle's own Table-1 map."""
    if mat.n_bath == 0:
        return None, None, None
    if mat.form is not None:
        return closed_form.table1_bath(mat.form, mat.omega0, mat.gamma0, mat.n_bath, mat.width,
                                       mat.bath_gamma, mat.dephasing)
    return (np.asarray(mat.omega_j, np.float64), np.asarray(mat.gamma_j, np.float64),
            np.asarray(mat.k_j, np.float64))


class Oracle:
    """One FP64 grid on the CPU, set up from a workload description.  A problem with Bloch phases
    (problem.bloch) holds two grids, the real and imaginary parts of the complex fields (gi is the
    imaginary part's grid); fields, polarizations and bath coordinates then read back complex, the
    flux is that of the complex fields and the energies are the sums over both parts."""

    def __init__(self, problem, closures: Optional[Dict[int, dict]] = None):
        self.p = problem
        self._keep = []
        self.gi = None
        self.g = self._make(problem, closures, 0)
        if problem.bloch is not None:
            if closures:
                raise ValueError("oracle: learned closures on Bloch grids are not supported")
            self.gi = self._make(problem, None, 1)
            ph = np.ascontiguousarray(problem.bloch, np.float64)
            if lib().or_pair_bloch(self.g, self.gi, ph) != 0:
                raise ValueError("oracle: bad Bloch phases (periodic axes only)")

    def _make(self, problem, closures, part: int):
        """One grid with the problem's set-up; part 1 (imaginary part of a Bloch grid) takes the
        imaginary parts of the source profiles (sources without one are real and drive part 0 only)."""
        L = lib()
        n = problem.n
        g = L.or_create(problem.ndim, n[0], n[1], n[2], problem.courant)
        if not g:
            raise ValueError("oracle: bad grid")
        for a in range(problem.ndim):
            L.or_set_boundary(g, a, int(problem.bc[a]), int(problem.pml_cells[a]), float(problem.pml_R0))
        self._setup(g, problem, closures, part)
        return g

    def _setup(self, g, problem, closures, part):
        L = lib()
        closures = closures or {}
        for mi, m in enumerate(problem.materials):
            lo, hi = _box(m.box)
            kind = type(m).__name__
            if kind == "Dielectric":
                rc = L.or_add_dielectric(g, lo, hi, m.eps_inf)
            elif kind == "Drude":
                rc = L.or_add_drude(g, lo, hi, m.omega_p, m.gamma, m.eps_inf)
            elif kind == "LorentzBath":
                sig = None if m.sigma_cells is None else np.ascontiguousarray(m.sigma_cells, np.float64).ravel()
                self._keep.append(sig)
                if mi in closures:
                    cl = closures[mi]
                    w = np.ascontiguousarray(cl["weights"], np.float64)
                    s = np.ascontiguousarray(cl["scales"], np.float64)
                    rc = L.or_add_closure(g, lo, hi, m.omega0, m.gamma0, m.eps_inf, _ptr(sig), m.sigma,
                                          float(cl["sum_kc"]), int(cl["width"]), w, s)
                else:
                    wj, gj, kj = bath_arrays(m)
                    self._keep += [wj, gj, kj]
                    rc = L.or_add_lorentz_bath(g, lo, hi, m.omega0, m.gamma0, m.eps_inf, _ptr(sig), m.sigma,
                                               m.n_bath, _ptr(wj), _ptr(gj), _ptr(kj))
                    if rc == 0 and m.kT:
                        rc = L.or_set_bath_thermal(g, mi, float(m.kT), int(m.noise_seed))
                    if rc == 0 and m.anharmonic is not None:
                        lam = np.ascontiguousarray(m.anharmonic, np.float64)
                        rc = L.or_set_bath_anharmonic(g, mi, lam)
            elif kind == "MultiPole":
                kinds = np.array([{"lorentz": 0, "drude": 1}[k] for k in m.kinds], np.int32)
                rc = L.or_add_multipole(g, lo, hi, m.eps_inf, len(kinds), kinds,
                                        np.ascontiguousarray(m.omega, np.float64), np.ascontiguousarray(m.gamma, np.float64),
                                        np.ascontiguousarray(m.sigma, np.float64))
            else:
                raise TypeError(kind)
            if rc != 0:
                raise ValueError(f"oracle: material {mi} rejected")
        for s in problem.sources:
            lo, hi = _box(s.box)
            pr = s.profile if part == 0 else s.profile_im
            if part == 1 and pr is None:
                continue
            prof = None if pr is None else np.ascontiguousarray(pr, np.float64).ravel()
            self._keep.append(prof)
            if L.or_add_source(g, s.comp, lo, hi, s.omega_c, s.width, s.amplitude, _ptr(prof)) < 0:
                raise ValueError("oracle: bad source")
        for d in problem.dfts:
            lo, hi = _box(d.box)
            om = np.ascontiguousarray(d.omega, np.float64)
            if L.or_add_dft(g, d.axis, lo, hi, len(om), om) < 0:
                raise ValueError("oracle: bad dft")
        for e in problem.energies:
            lo, hi = _box(e.box)
            if L.or_add_energy(g, lo, hi, e.every) < 0:
                raise ValueError("oracle: bad energy monitor")

    def __del__(self):
        for name in ("g", "gi"):
            g = getattr(self, name, None)
            if g:
                lib().or_destroy(g)
                setattr(self, name, None)

    def _both(self, fn):
        """fn(grid) of the real part, + 1j fn(grid) of the imaginary part on a Bloch grid"""
        v = fn(self.g)
        return v if self.gi is None else v + 1j * fn(self.gi)

    def step(self, n: int):
        lib().or_step(self.g, int(n))

    @property
    def steps_done(self) -> int:
        return lib().or_get_step(self.g)

    def field(self, comp: int) -> np.ndarray:
        def one(g):
            out = np.zeros(self.p.cells, np.float64)
            lib().or_get_field(g, comp, out)
            return out.reshape(self.p.n)
        return self._both(one)

    def set_field(self, comp: int, values: np.ndarray):
        lib().or_set_field(self.g, comp, np.ascontiguousarray(np.real(values), np.float64).ravel())
        if self.gi is not None:
            lib().or_set_field(self.gi, comp, np.ascontiguousarray(np.imag(values), np.float64).ravel())

    def polarization(self, mi: int, comp: int, level: int = 0) -> np.ndarray:
        m = self.p.materials[mi]
        nc = int(np.prod([m.box[1][a] - m.box[0][a] for a in range(3)]))

        def one(g):
            out = np.zeros(nc, np.float64)
            if lib().or_get_P(g, mi, comp, level, out) != 0:
                raise ValueError("no polarization")
            return out
        return self._both(one)

    def pole(self, mi: int, comp: int, pole: int, level: int = 0) -> np.ndarray:
        """Polarization of one term of a multi-term material."""
        m = self.p.materials[mi]
        nc = int(np.prod([m.box[1][a] - m.box[0][a] for a in range(3)]))

        def one(g):
            out = np.zeros(nc, np.float64)
            if lib().or_get_P_pole(g, mi, comp, level, pole, out) != 0:
                raise ValueError("no such term")
            return out
        return self._both(one)

    def set_pole(self, mi: int, comp: int, pole: int, level: int, values: np.ndarray):
        if lib().or_set_P_pole(self.g, mi, comp, level, pole, np.ascontiguousarray(values, np.float64).ravel()) != 0:
            raise ValueError("no such term")

    def bath(self, mi: int, comp: int, level: int = 0) -> np.ndarray:
        m = self.p.materials[mi]
        nc = int(np.prod([m.box[1][a] - m.box[0][a] for a in range(3)]))

        def one(g):
            out = np.zeros(m.n_bath * nc, np.float64)
            if lib().or_get_Y(g, mi, comp, level, out) != 0:
                raise ValueError("no bath")
            return out.reshape(m.n_bath, nc)
        return self._both(one)

    def set_polarization(self, mi: int, comp: int, level: int, values: np.ndarray):
        if lib().or_set_P(self.g, mi, comp, level, np.ascontiguousarray(values, np.float64).ravel()) != 0:
            raise ValueError("no polarization")

    def set_bath(self, mi: int, comp: int, level: int, values: np.ndarray):
        if lib().or_set_Y(self.g, mi, comp, level, np.ascontiguousarray(values, np.float64).ravel()) != 0:
            raise ValueError("no bath")

    @staticmethod
    def philox(counter, key) -> np.ndarray:
        """The oracle's own Philox4x32-10 on one counter (4 words) and key (2 words)."""
        out = np.zeros(4, np.uint32)
        lib().or_philox(np.ascontiguousarray(counter, np.uint32), np.ascontiguousarray(key, np.uint32), out)
        return out

    def drive(self, mi: int, comp: int, e_seq: np.ndarray) -> np.ndarray:
        """Advance material mi alone under a prescribed E sequence; returns P of its first cell."""
        e = np.ascontiguousarray(e_seq, np.float64)
        out = np.zeros(len(e), np.float64)
        if lib().or_drive_material(self.g, mi, comp, e, len(e), out) != 0:
            raise ValueError("cannot drive")
        return out

    def hidden(self, mi: int, comp: int) -> np.ndarray:
        m = self.p.materials[mi]
        nc = int(np.prod([m.box[1][a] - m.box[0][a] for a in range(3)]))
        out = np.zeros(4 * nc, np.float64)
        if lib().or_get_hidden(self.g, mi, comp, out) != 0:
            raise ValueError("no closure")
        return out.reshape(nc, 4)

    def flux(self, mid: int, raw: bool = False):
        d = self.p.dfts[mid]
        nf = len(d.omega)
        out = np.zeros(nf, np.float64)
        npts = int(np.prod([d.box[1][a] - d.box[0][a] for a in range(3)]))
        r = np.zeros(4 * npts * nf * 2, np.float64) if raw else None
        lib().or_get_dft(self.g, mid, out, _ptr(r))
        if raw:
            rr = r.reshape(4, npts, nf, 2)
            tr = rr[..., 0] + 1j * rr[..., 1]
            if self.gi is not None:   # transforms of the complex fields: real part's + 1j * imaginary part's
                ri = np.zeros(4 * npts * nf * 2, np.float64)
                lib().or_get_dft(self.gi, mid, np.zeros(nf, np.float64), _ptr(ri))
                ri = ri.reshape(4, npts, nf, 2)
                tr = tr + 1j * (ri[..., 0] + 1j * ri[..., 1])
            return out, tr
        return out

    def energy(self, mid: int) -> np.ndarray:
        """[field, polarization, bath] per sample (summed over both parts of a Bloch grid)"""
        tot = None
        for g in (self.g, self.gi):
            if g is None:
                continue
            n = lib().or_energy_count(g, mid)
            out = np.zeros(3 * max(n, 0), np.float64)
            if n > 0:
                lib().or_get_energy(g, mid, out)
            tot = out.reshape(-1, 3) if tot is None else tot + out.reshape(-1, 3)
        return tot


def run(problem, steps: Optional[int] = None, closures=None) -> Oracle:
    o = Oracle(problem, closures=closures)
    o.step(problem.steps if steps is None else steps)
    return o
