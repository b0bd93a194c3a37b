"""The 1D Fabry-Perot cavity of the Appendix on the GPU (FP64): transmission spectra of the cavity
filled with the plain Lorentz slab and with Lorentz-Bath slabs (Lorentzian and uniform bath forms of
Table 1), against the oracle, and the behaviour Sec. IV.B reports at the larger coupling: the
Lorentz-Bath polaritons transmit far more than the Lorentz ones, with the same Rabi splitting.

Parameters (Appendix, angular units c / dx with dx = 0.01 um): n = 10 mirrors 0.02 um thick, 1 um
apart, slab filling the cavity, nu0 = 1 um^-1, sigma = 0.02; Lorentz gamma / 2 pi = 0.04; bath
gamma0 / 2 pi = 0.0004, dephasing 0.99 gamma (reading of the printed value), gamma_b / 2 pi = 0.0004,
bath window omega0 +- 5 gamma.  The library holds at most 64 bath modes per cell, so N_b = 64 stands
in for the paper's 100.
"""
import numpy as np
import pytest

from fdtdb_inputs.problem import PERIODIC, PML, DftFlux, Drude, LorentzBath, Problem, Source, box

pytestmark = pytest.mark.gpu

DX = 0.01
N, M0, D, T = 600, 250, 100, 2
STEPS = 160000


def nu2w(nu):
    return 2 * np.pi * nu * DX


NU = np.linspace(0.6, 1.4, 801)


def problem(slab):
    p = Problem(name="fp-appendix", ndim=1, n=(N, 1, 1), bc=(PML, PERIODIC, PERIODIC), pml_cells=(40, 0, 0),
                dtype="f64", steps=STEPS)
    if slab is not None:
        p.materials += [Drude(box((M0 - T, M0)), omega_p=0.0, gamma=0.0, eps_inf=100.0), slab,
                        Drude(box((M0 + D, M0 + D + T)), omega_p=0.0, gamma=0.0, eps_inf=100.0)]
    p.sources.append(Source(comp=2, box=box((100, 101)), omega_c=nu2w(1.0), width=nu2w(1.2)))
    p.dfts.append(DftFlux(0, box((N - 150, N - 149)), nu2w(NU)))
    return p


def slabs(sig=0.02):
    G = nu2w(0.04)
    out = {"lorentz": LorentzBath(box((M0, M0 + D)), omega0=nu2w(1.0), gamma0=G, eps_inf=1.0, sigma=sig)}
    for form in ("lorentzian", "uniform"):
        out[form] = LorentzBath(box((M0, M0 + D)), omega0=nu2w(1.0), gamma0=nu2w(0.0004), eps_inf=1.0, sigma=sig,
                                n_bath=64, form=form, width=10 * G, bath_gamma=nu2w(0.0004), dephasing=0.99 * G)
    return out


def gpu_flux(p):
    from paper_2505_23963_amd import Grid
    print(f"[gpu] {p.name} {len(p.materials)} materials, {STEPS} steps", flush=True)
    g = Grid(p, graph_chunk=128)
    g.step(STEPS)
    return g.flux(0)


def test_fabry_perot_lorentz_bath_vs_lorentz(oracle_lib):
    empty = gpu_flux(problem(None))
    T = {k: gpu_flux(problem(s)) / empty for k, s in slabs().items()}
    # parity with the oracle on the Lorentzian-bath cavity (FP64 over 160 000 steps)
    fo = oracle_lib.run(problem(slabs()["lorentzian"])).flux(0)
    fg = T["lorentzian"] * empty
    assert np.max(np.abs(fg - fo)) <= 1e-9 * np.max(np.abs(fo))
    lo, up = (NU > 0.85) & (NU < 0.97), (NU > 1.03) & (NU < 1.15)
    peak = {k: (v[lo].max(), v[up].max()) for k, v in T.items()}
    print("[gpu] polariton peak transmission (lower, upper):",
          {k: (round(a, 4), round(b, 4)) for k, (a, b) in peak.items()}, flush=True)
    # Sec. IV.B: with the bath the polaritons are much brighter than with the equally broad Lorentz line
    for form in ("lorentzian", "uniform"):
        assert min(peak[form]) > 5 * max(peak["lorentz"]), form
    # the Rabi splitting of the transmission-weighted polariton centres is about omega0 sqrt(sigma)
    v = T["lorentzian"]
    c_lo = np.sum(NU[lo] * v[lo]) / np.sum(v[lo])
    c_up = np.sum(NU[up] * v[up]) / np.sum(v[up])
    assert abs((c_up - c_lo) - np.sqrt(0.02)) < 0.1 * np.sqrt(0.02), (c_lo, c_up)
