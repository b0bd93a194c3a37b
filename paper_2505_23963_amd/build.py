"""Build libfdtdb.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfdtdb.so")
SOURCES = ["fdtdb_kernels.hip", "fdtdb_runtime.hip", "fdtdb_batch.hip", "fdtdb_train.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-pass-failed",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in proc.stdout.splitlines() if "packed-fp32-ops" not in l)
    return proc.returncode, out


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel (one hipcc per file), then link the library."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build", f"obj{os.getpid()}")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    jobs = []
    for s in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        jobs.append((obj, [hipcc, *compile_flags, "-c", "-o", obj, os.path.join(CSRC, s)]))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda j: _run(j[1], verbose), jobs))
    for (rc, out), (obj, _) in zip(results, jobs):
        if rc != 0:
            sys.stderr.write(out + "\n")
            raise RuntimeError(f"hipcc failed compiling {os.path.basename(obj)}")
    tmp = LIB + f".tmp{os.getpid()}"
    rc, out = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *(o for o, _ in jobs)], verbose)
    if rc != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError("hipcc failed linking libfdtdb.so")
    os.replace(tmp, LIB)
    for o, _ in jobs:
        os.remove(o)
    os.rmdir(objdir)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
