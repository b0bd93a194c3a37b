"""Writes config2_full_200.npz: sampled columns of the FP64 oracle's run of the full 3D planar-cavity
workload (256 x 256 x 512, N_b = 8, per-cell sigma) after 200 steps, for the GPU's full-size parity
test.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_config2_full_sample.py        (about 6 minutes on 8 cores, 16 GB)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from fdtdb_inputs import configs  # noqa: E402

STEPS = 200
NFREQ = 16
# sampled (x, y) columns: the four corners of the periodic plane and points spread over it
COLUMNS = np.array([(0, 0), (255, 0), (0, 255), (255, 255), (37, 201), (128, 128), (200, 63), (91, 17)],
                   dtype=np.int64)


def main():
    p = configs.config2_3d(steps=STEPS, nfreq=NFREQ)
    t0 = time.time()
    o = oracle.Oracle(p)
    for done in range(0, STEPS, 20):
        o.step(20)
        print(f"oracle full size: {done + 20} steps, {time.time() - t0:.0f} s", flush=True)
    xs, ys = COLUMNS[:, 0], COLUMNS[:, 1]
    fields = np.stack([o.field(c)[xs, ys, :] for c in range(6)])                     # [6][ncol][512]
    lb = p.materials[1]
    nz = lb.box[1][2] - lb.box[0][2]
    pol = np.stack([o.polarization(1, c, 0).reshape(256, 256, nz)[xs, ys, :] for c in range(3)])
    bath = np.stack([o.bath(1, c, 0).reshape(lb.n_bath, 256, 256, nz)[:, xs, ys, :] for c in range(3)])
    norms = np.array([np.linalg.norm(o.field(c)) for c in range(6)])
    np.savez_compressed(os.path.join(HERE, "config2_full_200.npz"), steps=STEPS, nfreq=NFREQ, columns=COLUMNS,
                        fields=fields, polarization=pol, bath=bath, field_norms=norms, flux=o.flux(0))
    print(f"written in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
