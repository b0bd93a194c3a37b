"""What a learned closure with K = 4 hidden states can reach at best on the 2D workload's bath.

With identity activations the closure is a linear recurrent filter with four states, driven by E, P and
(P^{n+1/2} - P^{n-1/2})/dt; with tanh it is that filter to O(eps^2) after the eps carry-over.  Such a
filter turns the Lorentz medium's susceptibility into a rational function with two pole pairs in its bath
term (oracle.closed_form.k4_closure_susceptibility).  The explicit N_b = 64 bath has 64 pole pairs; the
transmission of a layer of the medium (the lattice transfer matrix, exact for the scheme) shows the
difference as a spectral error that no member of the class removes.
"""
import json
import os

import numpy as np

from fdtdb_inputs.problem import freq_grid
from oracle.closed_form import (chi_discrete, k4_closure_best_error, lattice_transmission,
                                lattice_transmission_uniform, table1_bath)

HERE = os.path.dirname(os.path.abspath(__file__))
DT = 0.5


def test_uniform_layer_transmission_equals_the_stack_recurrence():
    """The Chebyshev form of a uniform layer equals the node-by-node lattice recurrence (P7's transfer
    matrix), from one cell to a layer so absorbing that the recurrence needs rescaling."""
    w = np.linspace(0.5, 1.5, 201)
    wj, gj, kj = table1_bath("lorentzian", 1.0, 0.001, 64, 0.4, 0.4 / 63 / 2, 0.02)
    chi = chi_discrete(w, DT, 1.0, 0.001, 0.05, wj, gj, kj)
    for L in (1, 2, 9, 300):
        a = lattice_transmission(w, DT, np.full(L, 1.2), np.tile(chi, (L, 1)))
        b = lattice_transmission_uniform(w, DT, 1.2, chi, L)
        assert np.max(np.abs(a - b)) < 1e-12, L


def test_the_4_state_class_holds_a_two_mode_bath():
    """Two bath modes are four states: the fit reproduces that bath's transmission exactly (so the class and
    the search are wide enough for what four states can represent)."""
    w = freq_grid(256)
    wj, gj, kj = np.array([0.95, 1.08]), np.array([0.02, 0.03]), np.array([0.08, 0.12])
    err, _ = k4_closure_best_error(w, DT, 1.0, 0.001, 0.05, wj, gj, kj, 256, starts=3)
    assert err < 1e-6, err


def test_no_4_state_linear_closure_reaches_1e3_on_the_2d_workload_bath():
    """The Lorentzian-form N_b = 64 bath of the 2D learned-closure workload, in a layer as thick as its patch
    (1024 cells): the best 4-state linear closure found leaves a spectral error of about 6e-2, sixty times
    the 1e-3 target (tests/golden/closure_bound_k4.json, written by make_closure_bound.py, holds the value)."""
    import sys
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_closure_bound
    err = make_closure_bound.compute()
    stored = json.load(open(os.path.join(HERE, "golden", "closure_bound_k4.json")))["best_spectral_error"]
    print(f"best 4-state linear closure: spectral error {err:.3e}", flush=True)
    assert abs(err - stored) < 1e-6 * stored
    assert err > 1e-3 * 30
