"""FP32 parity measure shared by the GPU parity tests.

FP32 state is compared with the FP64 oracle field by field: the vector E (its active components
together), the vector H, and each Lorentz-Bath material's polarization P and bath coordinates Y (all
components, the newest level).  The error of a field at a checkpoint is ||x_gpu - x_oracle||_2
divided by the largest norm the oracle's field had up to then, sampled every 50 steps (the field's scale
over the run).  Each component is held to the same bar against the same scale.  Two properties of FP32
storage make the scale over the run, and not the field at the compared step, the measure:

* the storage rounds each stored word to 2^-24 of its value, so a component fed only by transverse
  differences of a much larger one (a field driven by diffraction) receives rounding noise of the
  large component's size; and
* rounding noise deposited in the Yee scheme's static (curl-free) modes stays where it is after a pulse
  has left through the absorbing layers, while the field itself decays.

Each component's error against its own norm at the compared step is printed beside it.
"""
from __future__ import annotations

import numpy as np

TOL_F32 = 1e-5


def field_groups(p, closures=()):
    """[(name, getter(grid_or_oracle) -> list of component arrays)] of the fields compared (materials
    whose bath a learned closure replaces have no bath coordinates)."""
    from fdtdb_inputs.problem import active_components
    e, h = active_components(p.ndim)
    out = [("E", lambda x, e=e: [x.field(c) for c in e]), ("H", lambda x, h=h: [x.field(c) for c in h])]
    for mi, m in enumerate(p.materials):
        if type(m).__name__ == "MultiPole":
            for q, kind in enumerate(m.kinds):
                if kind == "drude":      # the GPU keeps a Drude term's increment P^{n+1/2} - P^{n-1/2}
                    out.append((f"V{mi}.{q}", lambda x, mi=mi, q=q, e=e: [term_increment(x, mi, c, q) for c in e]))
                else:
                    out.append((f"P{mi}.{q}", lambda x, mi=mi, q=q, e=e: [x.pole(mi, c, q, 0) for c in e]))
            continue
        if type(m).__name__ != "LorentzBath":
            continue
        out.append((f"P{mi}", lambda x, mi=mi, e=e: [x.polarization(mi, c, 0) for c in e]))
        if m.n_bath and mi not in closures:
            out.append((f"Y{mi}", lambda x, mi=mi, e=e: [x.bath(mi, c, 0) for c in e]))
    return out


def term_increment(x, mi, c, q):
    """P^{n+1/2} - P^{n-1/2} of term q of a multi-term material: the oracle keeps both levels, the GPU library
    keeps a Drude term's increment itself (its level 0)."""
    if type(x).__module__.split(".")[0] == "oracle":
        return x.pole(mi, c, q, 0) - x.pole(mi, c, q, 1)
    return x.pole(mi, c, q, 0)


class Lockstep:
    """Advance a GPU object and the oracle together and measure every field at each checkpoint; the
    oracle's field norms (the fields' scale) are taken every `norm_every` steps in between, so that
    the scale sees the pulse at its peak."""

    def __init__(self, gpu, orc, p, groups=None, closures=(), norm_every: int = 50):
        self.g, self.o, self.p = gpu, orc, p
        self.groups = groups or field_groups(p, closures)
        self.norm_every = norm_every
        self.peak = {}
        self.rows = []

    def _track_norms(self):
        for name, get in self.groups:
            n = float(np.sqrt(sum(np.linalg.norm(r) ** 2 for r in get(self.o))))
            self.peak[name] = max(self.peak.get(name, 0.0), n)

    def run(self, total: int, every: int):
        done = 0
        while done < total:
            n = min(every, total - done)
            self.g.step(n)
            k = 0
            while k < n:
                m = min(self.norm_every, n - k)
                self.o.step(m)
                k += m
                if k < n:
                    self._track_norms()
            done += n
            self.g.synchronize()
            self.rows.append((done, self.measure()))
            print(f"  step {done}: " + "  ".join(f"{k} {v['err']:.2e}" for k, v in self.rows[-1][1].items()),
                  flush=True)
        return self

    def measure(self):
        out = {}
        for name, get in self.groups:
            ref, got = get(self.o), get(self.g)
            n = float(np.sqrt(sum(np.linalg.norm(r) ** 2 for r in ref)))
            self.peak[name] = max(self.peak.get(name, 0.0), n)
            scale = self.peak[name] if self.peak[name] > 0 else 1.0
            d = [float(np.linalg.norm(np.asarray(a) - np.asarray(b))) for a, b in zip(got, ref)]
            own = [di / max(float(np.linalg.norm(r)), 1e-300) for di, r in zip(d, ref)]
            out[name] = {"err": float(np.sqrt(sum(x * x for x in d))) / scale,
                         "comp": [x / scale for x in d], "own": own, "norm": n, "peak": self.peak[name]}
        return out

    def worst(self):
        """Largest field error and largest component error (both against the field's scale) over all
        checkpoints."""
        e = max(v["err"] for _, r in self.rows for v in r.values())
        c = max(max(v["comp"]) for _, r in self.rows for v in r.values())
        return e, c

    def report(self):
        step, last = self.rows[-1]
        for k, v in last.items():
            print(f"  {k} at step {step}: {v['err']:.3e} of its scale (norm {v['norm']:.3e}, peak {v['peak']:.3e}); "
                  f"components vs own norm " + ", ".join(f"{x:.2e}" for x in v["own"]), flush=True)


def flux_errors(flux_gpu, flux_orc, raw_orc):
    """(relative L2 of the flux spectrum, its error against the flux's cancellation scale).

    The scale at each frequency is sum_p |E~_t1 H~_t2| + |E~_t2 H~_t1| from the oracle's accumulators:
    inside a closed cavity the net flux is a small difference of such products, so its relative error
    measures the cancellation more than the arithmetic."""
    d = np.asarray(flux_gpu) - np.asarray(flux_orc)
    rel = float(np.linalg.norm(d) / max(np.linalg.norm(flux_orc), 1e-300))
    e1, e2, h1, h2 = raw_orc
    sc = np.sum(np.abs(e1 * h2) + np.abs(e2 * h1), axis=0)
    return rel, float(np.linalg.norm(d) / max(np.linalg.norm(sc), 1e-300))
