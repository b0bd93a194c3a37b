"""Seeded synthetic workloads for the FDTD-Bath time step.

Random numbers (Philox4x32-10) and plain-data problem descriptions only; this
package holds none of the update arithmetic.  The GPU library binding, the
tests, the benchmark and the oracle all read their inputs from here.
"""
from .philox import Stream, philox4x32  # noqa: F401
from .problem import *  # noqa: F401,F403
from . import configs  # noqa: F401
