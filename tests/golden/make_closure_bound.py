"""Writes closure_bound_k4.json: the smallest spectral error any 4-state linear closure was found to reach
(oracle.closed_form.k4_closure_best_error, six seeded starts) on the bath of the 2D learned-closure
workload (Lorentzian form, N_b = 64, width 0.4, dephasing 0.02, gamma_b = width / (N_b - 1) / 2,
omega0 = 1, gamma0 = 0.001, sigma = 0.05), for a layer as thick as the workload's patch (1024 cells) on
the workload's 256-frequency grid.  Calls only the oracle's closed forms.

    python tests/golden/make_closure_bound.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from fdtdb_inputs.problem import freq_grid  # noqa: E402
from oracle.closed_form import k4_closure_best_error, table1_bath  # noqa: E402

BATH = dict(form="lorentzian", omega0=1.0, gamma0=0.001, nb=64, width=0.4, bath_gamma=0.4 / 63 / 2, dephasing=0.02)
SIGMA, LAYER, STARTS, SEED = 0.05, 1024, 6, 0


def compute():
    wj, gj, kj = table1_bath(BATH["form"], BATH["omega0"], BATH["gamma0"], BATH["nb"], BATH["width"],
                             BATH["bath_gamma"], BATH["dephasing"])
    err, _ = k4_closure_best_error(freq_grid(256), 0.5, BATH["omega0"], BATH["gamma0"], SIGMA, wj, gj, kj, LAYER,
                                   starts=STARTS, seed=SEED)
    return err


def main():
    err = compute()
    out = {"bath": BATH, "sigma": SIGMA, "layer_cells": LAYER, "frequencies": "256 on [0.5, 1.5]", "starts": STARTS,
           "seed": SEED, "best_spectral_error": err}
    json.dump(out, open(os.path.join(HERE, "closure_bound_k4.json"), "w"), indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
