"""Learned bath closure: record, train, validate, and the fallback decision.

Host orchestration of C-ABI calls only; every arithmetic step (the explicit solver that produces
the training trajectories, the FP64 bath-force targets, forward/backward passes, Adam, closure
inference) runs in libfdtdb.so.

Recipe (training is in the closure's linear regime because the bath force is a linear causal
filter of the polarization history, eq:EOM_LorentzBath-2):
  1. run the explicit Lorentz-Bath solver and record E^{n+1/2} and P^{n+3/2} at chosen cells;
  2. train with identity activations (the network is then a 4-state linear filter) by truncated
     BPTT + Adam on the GPU;
  3. carry the weights into the tanh network by eps scaling (same function to O(eps^2));
  4. validate against the explicit bath on a run of the target geometry; if the spectral error
     exceeds the tolerance, keep the explicit bath (fallback).
"""
from __future__ import annotations

import time
from typing import Optional

import numpy as np

from .fdtdb import Grid, Trainer, bath_params, closure_weights


def bath_arrays(mat):
    if mat.form is not None:
        return bath_params(mat.form, mat.omega0, mat.gamma0, mat.n_bath, mat.width, mat.bath_gamma, mat.dephasing)
    return (np.asarray(mat.omega_j, np.float64), np.asarray(mat.gamma_j, np.float64),
            np.asarray(mat.k_j, np.float64))


def record(problem, mi: int, comp: int, cells, nsteps: int, stream: Optional[int] = None):
    """Run the explicit solver for nsteps from rest; return the (E, P) records [nsteps][cells]."""
    g = Grid(problem, stream=stream)
    pid = g.add_probe(mi, comp, cells, nsteps)
    g.step(nsteps)
    return g.probe_data(pid)


def train(E, P, dt: float, mat, init: dict, window: int = 64, epochs: int = 600, lr: float = 3e-3,
          lr_decay: float = 0.99, eps: float = 1e-4, stream: Optional[int] = None) -> dict:
    """Train a closure on records of the explicit bath of `mat`; returns weights (tanh network),
    scales, the final loss of the linear stage, the loss of the tanh network and the loss curve."""
    wj, gj, kj = bath_arrays(mat)
    T, N = E.shape
    tr = Trainer(N, T, window, dt, wj, gj, kj, activation="identity", stream=stream)
    tr.load(E, P)
    tr.set_weights(closure_weights(init))
    t0 = time.perf_counter()
    curve = tr.train(epochs, lr, lr_decay)
    t_train = time.perf_counter() - t0
    lin, _ = tr.loss_grad()
    tr.set_activation("tanh", eps)
    tl, _ = tr.loss_grad()
    return {"weights": tr.weights(), "scales": tr.scales(), "loss_linear": lin, "loss_tanh": tl, "curve": curve,
            "train_seconds": t_train, "windows_per_epoch": T // window, "trajectories": N}


def spectral_error(flux, ref) -> float:
    """max |flux - ref| / max |ref| over the monitor's frequencies."""
    return float(np.max(np.abs(flux - ref)) / np.max(np.abs(ref)))


def validate(problem, mi: int, closure: dict, steps: int, monitor: int = 0, tol: float = 1e-3,
             stream: Optional[int] = None):
    """Run the explicit and the closure grid for `steps`; returns (use_closure, spectral error,
    explicit flux, closure flux).  use_closure is False (fallback to the explicit bath) when the
    spectral error exceeds tol."""
    ge = Grid(problem, stream=stream)
    ge.step(steps)
    fe = ge.flux(monitor)
    del ge
    gc = Grid(problem, stream=stream, closures={mi: {"weights": closure["weights"], "scales": closure["scales"]}})
    gc.step(steps)
    fc = gc.flux(monitor)
    err = spectral_error(fc, fe)
    return err <= tol, err, fe, fc
