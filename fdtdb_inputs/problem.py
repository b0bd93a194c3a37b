"""Plain-data description of an FDTD-Bath workload.

A Problem lists the grid, its boundaries, the material boxes, the sources and
the monitors.  Both the GPU library binding and the oracle driver consume it;
it holds numbers only (no update arithmetic).  Boxes are half-open cell ranges
(lo, hi) over the three axes (x, y, z); unused axes of 1D/2D grids have the
range (0, 1).

Conventions (shared vocabulary, not arithmetic): c = eps0 = mu0 = 1, dx = 1,
dt = courant * dx, angular frequencies.  1D grids run along x with (Ez, Hy);
2D grids are the x-y plane with (Ez, Hx, Hy); 3D grids carry all six
components, z fastest in memory.  Field component ids: 0..2 = Ex, Ey, Ez;
3..5 = Hx, Hy, Hz.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

Box = Tuple[Tuple[int, int, int], Tuple[int, int, int]]

PML, PERIODIC, CLOSED = 0, 1, 2


def box(x: Tuple[int, int], y: Tuple[int, int] = (0, 1), z: Tuple[int, int] = (0, 1)) -> Box:
    return ((x[0], y[0], z[0]), (x[1], y[1], z[1]))


def box_cells(b: Box) -> int:
    return int(np.prod([b[1][a] - b[0][a] for a in range(3)]))


@dataclass
class Dielectric:
    box: Box
    eps_inf: float


@dataclass
class Drude:
    box: Box
    omega_p: float
    gamma: float
    eps_inf: float


@dataclass
class LorentzBath:
    """Lorentz polarization coupled to n_bath explicit bath oscillators (n_bath = 0: plain Lorentz).

    Either give omega_j/gamma_j/k_j explicitly, or give a bath form
    ('uniform' | 'lorentzian' | 'gaussian') with width, bath_gamma and
    dephasing, which each side maps to (omega_j, gamma_j, k_j) itself.
    """
    box: Box
    omega0: float
    gamma0: float
    eps_inf: float
    sigma: float = 0.0
    sigma_cells: Optional[np.ndarray] = None      # per cell of the box, C order (x, y, z)
    n_bath: int = 0
    omega_j: Optional[np.ndarray] = None
    gamma_j: Optional[np.ndarray] = None
    k_j: Optional[np.ndarray] = None
    form: Optional[str] = None
    width: float = 0.0
    bath_gamma: float = 0.0
    dephasing: float = 0.0
    # storage of the bath coordinates on the GPU: None (the state type), "f16" or "bf16" of Y * bath_scale
    bath_storage: Optional[str] = None
    bath_scale: float = 1.0
    # thermal bath: temperature kT (energy units; 0 = none) and the 64-bit seed of its noise
    kT: float = 0.0
    noise_seed: int = 0
    # anharmonic bath: quartic coefficient lambda_j of each mode (None = harmonic)
    anharmonic: Optional[np.ndarray] = None


@dataclass
class MultiPole:
    """A sum of Lorentz and Drude terms on one box: kinds[p] 'lorentz' (omega[p] = omega0, gamma[p], sigma[p])
    or 'drude' (omega[p] = omega_p, gamma[p]; sigma unused)."""
    box: Box
    eps_inf: float
    kinds: Sequence[str]
    omega: Sequence[float]
    gamma: Sequence[float]
    sigma: Sequence[float]


@dataclass
class Source:
    comp: int
    box: Box
    omega_c: float
    width: float
    amplitude: float = 1.0
    profile: Optional[np.ndarray] = None          # per cell of the box
    profile_im: Optional[np.ndarray] = None       # Bloch grids: imaginary part of a complex profile


@dataclass
class DftFlux:
    axis: int
    box: Box                                      # one cell thick along axis
    omega: np.ndarray


@dataclass
class EnergyMonitor:
    box: Box
    every: int


@dataclass
class Problem:
    name: str
    ndim: int
    n: Tuple[int, int, int]
    courant: float = 0.5
    bc: Tuple[int, int, int] = (PERIODIC, PERIODIC, PERIODIC)
    pml_cells: Tuple[int, int, int] = (0, 0, 0)
    pml_R0: float = 1e-8
    dtype: str = "f32"
    materials: List[object] = field(default_factory=list)
    sources: List[Source] = field(default_factory=list)
    dfts: List[DftFlux] = field(default_factory=list)
    energies: List[EnergyMonitor] = field(default_factory=list)
    steps: int = 100
    # Bloch phases phi_a = k_a n_a (radians) of the periodic axes: the fields become complex with
    # f(r + n_a e_a) = exp(i phi_a) f(r); None keeps real fields (plain periodic axes)
    bloch: Optional[Tuple[float, float, float]] = None

    @property
    def cells(self) -> int:
        return int(np.prod(self.n))

    @property
    def dt(self) -> float:
        return self.courant


def freq_grid(n: int, lo: float = 0.5, hi: float = 1.5) -> np.ndarray:
    """Uniform frequency grid with both endpoints."""
    return np.linspace(lo, hi, n)


def bath_grid(n: int, lo: float, hi: float) -> np.ndarray:
    """Bath frequencies evenly spaced with both endpoints (the paper's window)."""
    return np.linspace(lo, hi, n)


def active_components(ndim: int) -> Tuple[Sequence[int], Sequence[int]]:
    """(E components, H components) carried by a grid of this dimension."""
    if ndim == 1:
        return (2,), (4,)
    if ndim == 2:
        return (2,), (3, 4)
    return (0, 1, 2), (3, 4, 5)
